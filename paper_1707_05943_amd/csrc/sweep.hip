// The sweep's arithmetic around the network: the network's input encoding
// and the a-posteriori check of its P_e against FP64 solves on coarser grids
// (the estimate rests on the O(Delta^2) accuracy of the scheme's finite
// differences, Sec. 3, which the check verifies point by point).

#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "surrogate.h"

namespace {

// Encoding of instance b at sample p (8 channels): the incident packet
// phi(-a - sigma), sigma_p = 16 w p/(n-1), without its normalisation (real,
// imaginary; the packet's centre x0 = -a - 8w sits at sigma = 8w), then
// Gamma 2a / 10, k0 a / 2 pi, ln w / ln 5, Delta / 0.01, ln(Gamma T) / ln 1000
// (T the end of the P_e window) and p / (n-1).  par[b] = (w, k0, a, Gamma,
// Delta, T).
__global__ void k_encode(const double* __restrict__ par, int32_t n, float* __restrict__ x)
{
    const int64_t b = blockIdx.y;
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double* q = par + 6 * b;
    const double w = q[0], k0 = q[1], a = q[2], G = q[3], dl = q[4], T = q[5];
    const double pp = (double)p / (double)(n - 1);
    const double u = 8.0 - 16.0 * pp;
    const double env = exp(-0.25 * u * u);
    double s, c;
    sincos(k0 * w * u, &s, &c);
    float* o = x + ((int64_t)b * n + p) * 8;
    o[0] = (float)(env * c);
    o[1] = (float)(env * s);
    o[2] = (float)(G * 2.0 * a / 10.0);
    o[3] = (float)(k0 * a / (2.0 * M_PI));
    o[4] = (float)(log(w) / log(5.0));
    o[5] = (float)(dl / 0.01);
    o[6] = (float)(log(G * T) / log(1000.0));
    o[7] = (float)pp;
}

constexpr int CK_THREADS = 256;

// one workgroup per point.  With P_h = P + K h^2 in the scheme's asymptotic
// range, P2 - P_fine = (P4 - P2)(h2^2 - h0^2)/(h4^2 - h2^2) to leading order
// (`safety` multiplies that estimate), and |P8 - P4| / |P4 - P2| equals
// rho = (h8^2 - h4^2)/(h4^2 - h2^2); q is the observed ratio over rho.  A
// point outside the range (|q - 1| > ratio_tol) is accepted for neither
// path; inside it, for the network when dist + est <= tol and for the
// coarse solve alone when est <= tol.
__global__ __launch_bounds__(CK_THREADS) void k_check(const double* __restrict__ S, const double* __restrict__ P2,
                                                       const double* __restrict__ P4, const double* __restrict__ P8,
                                                       const double* __restrict__ h,
                                                       const int32_t* __restrict__ valid, int32_t n, double tol,
                                                       double safety, double ratio_tol, double* __restrict__ out,
                                                       int32_t* __restrict__ acc)
{
    __shared__ double red[4][CK_THREADS];
    const int64_t b = blockIdx.x;
    const double* s = S + b * n;
    const double* p2 = P2 + b * n;
    const double* p4 = P4 + b * n;
    const double* p8 = P8 + b * n;
    double d_s = 0.0, d_24 = 0.0, d_48 = 0.0, n2 = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += CK_THREADS) {
        const double e = s[i] - p2[i], f = p4[i] - p2[i], g = p8[i] - p4[i];
        d_s += e * e;
        d_24 += f * f;
        d_48 += g * g;
        n2 += p2[i] * p2[i];
    }
    red[0][threadIdx.x] = d_s;
    red[1][threadIdx.x] = d_24;
    red[2][threadIdx.x] = d_48;
    red[3][threadIdx.x] = n2;
    __syncthreads();
    for (int o = CK_THREADS / 2; o > 0; o >>= 1) {              // fixed-order tree
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double h0 = h[4 * b], h2 = h[4 * b + 1], h4 = h[4 * b + 2], h8 = h[4 * b + 3];
        const double nrm = sqrt(red[3][0]) > 1e-300 ? sqrt(red[3][0]) : 1e-300;
        const double d24 = sqrt(red[1][0]);
        const double dist = sqrt(red[0][0]) / nrm;
        const double wgt = (h2 * h2 - h0 * h0) / (h4 * h4 - h2 * h2);
        const double rho = (h8 * h8 - h4 * h4) / (h4 * h4 - h2 * h2);
        const double est = safety * fabs(wgt) * d24 / nrm;
        const double q = (sqrt(red[2][0]) / (d24 > 1e-300 ? d24 : 1e-300)) / rho;
        const int ok = valid[b] != 0 && isfinite(dist) && isfinite(est) && isfinite(q) && fabs(q - 1.0) <= ratio_tol;
        out[3 * b] = dist;
        out[3 * b + 1] = est;
        out[3 * b + 2] = q;
        acc[2 * b] = ok && dist + est <= tol;
        acc[2 * b + 1] = ok && est <= tol;
    }
}

}  // namespace

extern "C" int sur_encode(const double* d_par, int32_t B, int32_t n, float* d_x, void* hip_stream)
{
    if (!d_par || !d_x || B < 0 || n < 2) return SUR_EINVAL;
    // instances along the grid's y dimension, at most 65535 per launch
    for (int32_t b0 = 0; b0 < B; b0 += 65535) {
        const int32_t nb = B - b0 < 65535 ? B - b0 : 65535;
        hipLaunchKernelGGL(k_encode, dim3((unsigned)((n + 255) / 256), (unsigned)nb), dim3(256), 0,
                           (hipStream_t)hip_stream, d_par + (int64_t)6 * b0, n, d_x + (int64_t)b0 * n * 8);
        if (hipGetLastError() != hipSuccess) return SUR_EDEVICE;
    }
    return SUR_OK;
}

extern "C" int sur_check(const double* d_S, const double* d_P2, const double* d_P4, const double* d_P8,
                         const double* d_h, const int32_t* d_valid, int32_t B, int32_t n, double tol, double safety,
                         double ratio_tol, double* d_out, int32_t* d_acc, void* hip_stream)
{
    if (!d_S || !d_P2 || !d_P4 || !d_P8 || !d_h || !d_valid || !d_out || !d_acc || B < 0 || n < 1)
        return SUR_EINVAL;
    if (B == 0) return SUR_OK;
    hipLaunchKernelGGL(k_check, dim3((unsigned)B), dim3(CK_THREADS), 0, (hipStream_t)hip_stream, d_S, d_P2, d_P4,
                       d_P8, d_h, d_valid, n, tol, safety, ratio_tol, d_out, d_acc);
    return hipGetLastError() == hipSuccess ? SUR_OK : SUR_EDEVICE;
}
