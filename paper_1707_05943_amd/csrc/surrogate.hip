// Surrogate of the march: a one-dimensional Fourier neural operator (FNO)
// trained on the solver's outputs, with its forward and backward passes on
// bf16 matrix cores (MFMA 32x32x16, fp32 accumulation) and Adam in fp32.
//
// Network (n points, width C, `modes` Fourier modes, L layers, P hidden):
//   u0 = x W0 + b0                                   lift, x: (B, n, c_in)
//   for l < L:  X = F^T u_l  (DFT to the first `modes` modes, as a GEMM)
//               Y_m = X_m R_m  (complex C x C mixing per mode)
//               z_l = G Y + u_l W_l + b_l  (G: inverse DFT of the kept modes)
//               u_{l+1} = gelu(z_l)  (no activation after the last layer)
//   h = gelu(u_L W1 + b1),  y = h W2 + b2            projection, y: (B, n, c_out)
// Activations are (B, n, C) row-major; spectra (B, 2 modes, C) with rows
// 2m (real part) and 2m+1 (imaginary part).  Parameters are one fp32 array;
// every product reads fp32 and rounds to bf16 on its way into LDS.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "surrogate.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// batched GEMM: C[z] = alpha op(A[z]) op(B[z]) + beta C[z], fp32 in memory,
// bf16 operands, fp32 accumulation.  Tile 64 x 64 x 32, four waves, each
// wave one 32 x 32 block (two 32x32x16 MFMAs per k-tile).
// ---------------------------------------------------------------------------
constexpr int GB_M = 64, GB_N = 64, GB_K = 32, GB_LD = GB_K + 8;   // LDS rows padded by 16 bytes

struct GemmArgs {
    const float* A;
    const float* B;
    float* C;
    int M, N, K;
    int lda, ldb, ldc;
    long long sA, sB, sC;     // batch strides (elements)
    int transA, transB;
    float alpha, beta;
    int splits;               // split of K over blockIdx.z (1: none)
    float* part;              // splits > 1: raw products, (batch, splits, M, N)
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs a)
{
    __shared__ __bf16 As[GB_M][GB_LD];     // As[i][k]
    __shared__ __bf16 Bs[GB_N][GB_LD];     // Bs[j][k]
    const int z = blockIdx.z / a.splits, sp = blockIdx.z % a.splits;
    const float* A = a.A + z * a.sA;
    const float* B = a.B + z * a.sB;
    float* C = a.C + z * a.sC;
    const int i0 = blockIdx.y * GB_M, j0 = blockIdx.x * GB_N;
    // this split's share of K, in whole k-tiles
    const int ktiles = (a.K + GB_K - 1) / GB_K;
    const int per = (ktiles + a.splits - 1) / a.splits;
    const int kbeg = sp * per * GB_K;
    int kend = (sp + 1) * per * GB_K;
    if (kend > a.K) kend = a.K;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
    f32x16 acc;
    #pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    for (int k0 = kbeg; k0 < kend; k0 += GB_K) {
        // A tile: 64 x 32 values, 8 per thread; consecutive threads walk the
        // contiguous index of the stored matrix
        #pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = t + 256 * e;
            int ii, kk;
            if (!a.transA) { ii = idx >> 5; kk = idx & 31; } else { ii = idx & 63; kk = idx >> 6; }
            const int gi = i0 + ii, gk = k0 + kk;
            float v = 0.0f;
            if (gi < a.M && gk < kend) v = a.transA ? A[(long long)gk * a.lda + gi] : A[(long long)gi * a.lda + gk];
            As[ii][kk] = (__bf16)v;
        }
        #pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = t + 256 * e;
            int jj, kk;
            if (!a.transB) { jj = idx & 63; kk = idx >> 6; } else { jj = idx >> 5; kk = idx & 31; }
            const int gj = j0 + jj, gk = k0 + kk;
            float v = 0.0f;
            if (gj < a.N && gk < kend) v = a.transB ? B[(long long)gj * a.ldb + gk] : B[(long long)gk * a.ldb + gj];
            Bs[jj][kk] = (__bf16)v;
        }
        __syncthreads();
        // lane l supplies row (l mod 32) of A and column (l mod 32) of B at
        // k = 8 (l / 32) + v, v = 0..7, of each 16-wide k step; A and B use the
        // same k order, so the contraction is the same whatever order the
        // matrix core sums in
        const int r32 = lane & 31, kh = (lane >> 5) * 8;
        #pragma unroll
        for (int ks = 0; ks < GB_K; ks += 16) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&As[wi + r32][ks + kh]);
            const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Bs[wj + r32][ks + kh]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator r of lane l holds row 8 (r/4) + 4 (l/32) + r%4, column l mod 32
    #pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int ii = i0 + wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int jj = j0 + wj + (lane & 31);
        if (ii < a.M && jj < a.N) {
            if (a.splits > 1) {
                a.part[(((long long)z * a.splits + sp) * a.M + ii) * a.N + jj] = acc[r];
            } else {
                float* c = C + (long long)ii * a.ldc + jj;
                const float v = a.alpha * acc[r];
                *c = (a.beta != 0.0f) ? v + a.beta * *c : v;
            }
        }
    }
}

// sum of the split-K parts (fixed order), then alpha and beta
__global__ void k_gemm_reduce(GemmArgs a, int batch)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long mn = (long long)a.M * a.N;
    if (i >= mn * batch) return;
    const long long z = i / mn, e = i % mn;
    const int ii = (int)(e / a.N), jj = (int)(e % a.N);
    float s = 0.0f;
    for (int p = 0; p < a.splits; ++p) s += a.part[(z * a.splits + p) * mn + e];
    float* c = a.C + z * a.sC + (long long)ii * a.ldc + jj;
    const float v = a.alpha * s;
    *c = (a.beta != 0.0f) ? v + a.beta * *c : v;
}

// ---------------------------------------------------------------------------
// element-wise and reduction kernels
// ---------------------------------------------------------------------------
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_d(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// z = y + b[c] (kept), out = gelu(z) or z
__global__ void k_bias_act(float* y, const float* b, float* z_keep, long long rows, int C, int act)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * C) return;
    const float v = y[i] + b[i % C];
    if (z_keep) z_keep[i] = v;
    y[i] = act ? gelu(v) : v;
}

// dz = dout * gelu'(z)
__global__ void k_gelu_bwd(float* d, const float* z, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] *= gelu_d(z[i]);
}

// column sums of a rows x C matrix: per workgroup a chunk of rows, then a
// second pass over the chunks (fixed order, so the result is reproducible)
constexpr int CS_CHUNK = 256;
constexpr long long SPLIT_CAP = 1LL << 22;      // split-K scratch of the network's products (floats)
__global__ void k_colsum_part(const float* x, long long rows, int C, float* part)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const long long r0 = (long long)blockIdx.y * CS_CHUNK;
    long long r1 = r0 + CS_CHUNK;
    if (r1 > rows) r1 = rows;
    float s = 0.0f;
    for (long long r = r0; r < r1; ++r) s += x[r * C + c];
    part[(long long)blockIdx.y * C + c] = s;
}
__global__ void k_colsum_final(const float* part, int nchunk, int C, float* out, float beta)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float s = 0.0f;
    for (int k = 0; k < nchunk; ++k) s += part[(long long)k * C + c];
    out[c] = (beta != 0.0f) ? s + beta * out[c] : s;
}

// masked mean-squared error over (B, n, c_out) with per-channel weights:
// loss = sum w_o mask (y - t)^2 / count, dy = 2 w_o mask (y - t) / count;
// per-workgroup partial sums of the loss
__global__ void k_mse(const float* y, const float* t, const float* mask, const float* wo, long long n, int c_out,
                      float inv_count, float* dy, float* part)
{
    __shared__ float s[256];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        const float m = (mask ? mask[i] : 1.0f) * wo[i % c_out];
        const float e = y[i] - t[i];
        l = m * e * e * inv_count;
        dy[i] = 2.0f * m * e * inv_count;
    }
    s[threadIdx.x] = l;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
__global__ void k_sum(const float* part, int n, float* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int k = 0; k < n; ++k) s += part[k];
        *out = s;
    }
}

// Adam (bias-corrected moments), fp32
__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// forward DFT basis F (n x 2 modes): F[p][2m] = cos(2 pi m p / n),
// F[p][2m+1] = -sin(...); inverse G (n x 2 modes): G[p][2m] = c_m cos / n,
// G[p][2m+1] = -c_m sin / n with c_0 = 1, c_m = 2 (the kept modes of a real
// signal; the imaginary part of mode 0 drops out)
__global__ void k_dft_basis(float* F, float* G, int n, int modes)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * modes) return;
    const int p = (int)(i / modes), m = (int)(i % modes);
    const long long ph = ((long long)m * p) % n;          // exact angle index
    const double th = 2.0 * M_PI * (double)ph / (double)n;
    const double c = cos(th), s = sin(th);
    const double cm = (m == 0) ? 1.0 : 2.0;
    F[(long long)p * 2 * modes + 2 * m] = (float)c;
    F[(long long)p * 2 * modes + 2 * m + 1] = (float)(-s);
    G[(long long)p * 2 * modes + 2 * m] = (float)(cm * c / n);
    G[(long long)p * 2 * modes + 2 * m + 1] = (float)(-cm * s / n);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct sur_net {
    sur_cfg cfg;
    hipStream_t s;
    float* prm;              // caller's parameters (n_params)
    // offsets into prm
    long long oW0, ob0, oRr, oRi, oW, ob, oW1, ob1, oW2, ob2, n_params;
    // workspace views
    float *F, *G;            // DFT bases, n x 2 modes
    float* u;                // (L+1) activations (B, n, C)
    float* z;                // L pre-activations (B, n, C)
    float* X;                // L spectra (B, 2 modes, C)
    float* Y;                // spectrum after mixing (B, 2 modes, C), scratch
    float* zh;               // projection pre-activation (B, n, P)
    float* h;                // projection hidden (B, n, P)
    float* dA;               // gradient scratch (B, n, max(C, P))
    float* dB;               // gradient scratch (B, n, max(C, P))
    float* dX;               // (B, 2 modes, C)
    float* dY;               // (B, 2 modes, C)
    float* part;             // reduction partials
    float* split;            // split-K scratch (SPLIT_CAP floats)
    float* m1;               // Adam moments (n_params each)
    float* m2;
    int last_B;              // batch of the last forward (its activations are kept)
    char err[512];
};

static char g_serr[512];

static int sfail(sur_net* n, int code, const char* fmt, ...)
{
    char* dst = n ? n->err : g_serr;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

static long long al64(long long n) { return (n + 63) & ~63LL; }     // floats: 256-byte alignment

static int cfg_check(const sur_cfg* c, char* why, size_t n)
{
    if (!c || c->struct_size != sizeof(sur_cfg)) { snprintf(why, n, "cfg missing or struct_size mismatch"); return SUR_EINVAL; }
    if (c->n_points < 2 || c->c_in < 1 || c->width < 1 || c->modes < 1 || c->layers < 1 || c->proj < 1 ||
        c->c_out < 1 || c->max_batch < 1) {
        snprintf(why, n, "every size must be positive (n_points >= 2)");
        return SUR_EINVAL;
    }
    if (c->modes > c->n_points / 2) { snprintf(why, n, "modes must be <= n_points/2"); return SUR_EINVAL; }
    return SUR_OK;
}

struct Sizes {
    long long oW0, ob0, oRr, oRi, oW, ob, oW1, ob1, oW2, ob2, n_params;
    long long F, G, u, z, X, Y, zh, h, dA, dB, dX, dY, part, split, m1, m2, total;
};

static Sizes sizes_of(const sur_cfg* c)
{
    Sizes s;
    const long long C = c->width, M = c->modes, L = c->layers, P = c->proj;
    long long o = 0;
    s.oW0 = o; o += (long long)c->c_in * C;
    s.ob0 = o; o += C;
    s.oRr = o; o += L * M * C * C;
    s.oRi = o; o += L * M * C * C;
    s.oW = o; o += L * C * C;
    s.ob = o; o += L * C;
    s.oW1 = o; o += C * P;
    s.ob1 = o; o += P;
    s.oW2 = o; o += P * c->c_out;
    s.ob2 = o; o += c->c_out;
    s.n_params = o;
    const long long Bn = (long long)c->max_batch * c->n_points;
    const long long spec = (long long)c->max_batch * 2 * M * C;
    const long long wide = Bn * (C > P ? C : P);
    long long w = 0;
    s.F = w; w += al64((long long)c->n_points * 2 * M);
    s.G = w; w += al64((long long)c->n_points * 2 * M);
    s.u = w; w += al64((L + 1) * Bn * C);
    s.z = w; w += al64(L * Bn * C);
    s.X = w; w += al64(L * spec);
    s.Y = w; w += al64(spec);
    s.zh = w; w += al64(Bn * P);
    s.h = w; w += al64(Bn * P);
    s.dA = w; w += al64(wide);
    s.dB = w; w += al64(wide);
    s.dX = w; w += al64(spec);
    s.dY = w; w += al64(spec);
    const long long chunks = (Bn + CS_CHUNK - 1) / CS_CHUNK;
    const long long npart = chunks * (C > P ? C : P) > (Bn * c->c_out + 255) / 256 ? chunks * (C > P ? C : P)
                                                                                   : (Bn * c->c_out + 255) / 256;
    s.part = w; w += al64(npart + 64);
    s.split = w; w += SPLIT_CAP;
    s.m1 = w; w += al64(s.n_params);
    s.m2 = w; w += al64(s.n_params);
    s.total = w * 4;
    return s;
}

static int gemm(hipStream_t st, int transA, int transB, int M, int N, int K, float alpha, const float* A, int lda,
                long long sA, const float* B, int ldb, long long sB, float beta, float* C, int ldc, long long sC,
                int batch, float* split_ws = nullptr)
{
    if (M <= 0 || N <= 0 || batch <= 0) return SUR_OK;
    GemmArgs a;
    a.splits = 1;
    a.part = split_ws;
    // few output tiles over a long K: split K so that the chip has work
    const long long tiles = (long long)((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N) * batch;
    if (split_ws && tiles < 128 && K >= 8 * GB_K) {
        long long sp = 256 / tiles;
        const long long kt = (K + GB_K - 1) / GB_K;
        if (sp > kt / 4) sp = kt / 4;
        while (sp > 1 && sp * (long long)M * N * batch > SPLIT_CAP) --sp;
        if (sp > 1) a.splits = (int)sp;
    }
    a.A = A; a.B = B; a.C = C;
    a.M = M; a.N = N; a.K = K;
    a.lda = lda; a.ldb = ldb; a.ldc = ldc;
    a.sA = sA; a.sB = sB; a.sC = sC;
    a.transA = transA; a.transB = transB;
    a.alpha = alpha; a.beta = beta;
    dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, batch * a.splits);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, a);
    if (a.splits > 1) {
        const long long n = (long long)M * N * batch;
        hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, batch);
    }
    return hipGetLastError() == hipSuccess ? SUR_OK : SUR_EDEVICE;
}

static unsigned nblk(long long n, int th) { return (unsigned)((n + th - 1) / th); }

// out[c] (= or +=) column sums of x (rows x C)
static void colsum(sur_net* n, const float* x, long long rows, int C, float* out, float beta)
{
    const int chunks = (int)((rows + CS_CHUNK - 1) / CS_CHUNK);
    hipLaunchKernelGGL(k_colsum_part, dim3(nblk(C, 64), chunks), dim3(64), 0, n->s, x, rows, C, n->part);
    hipLaunchKernelGGL(k_colsum_final, dim3(nblk(C, 64)), dim3(64), 0, n->s, n->part, chunks, C, out, beta);
}

extern "C" {

int sur_sizes(const sur_cfg* cfg, int64_t* n_params, size_t* ws_bytes)
{
    char why[256];
    int rc = cfg_check(cfg, why, sizeof why);
    if (rc) return sfail(nullptr, rc, "%s", why);
    const Sizes s = sizes_of(cfg);
    if (n_params) *n_params = s.n_params;
    if (ws_bytes) *ws_bytes = (size_t)s.total;
    return SUR_OK;
}

int sur_init(const sur_cfg* cfg, float* d_params, void* d_ws, size_t bytes, void* hip_stream, sur_net** out)
{
    char why[256];
    if (!out) return sfail(nullptr, SUR_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = cfg_check(cfg, why, sizeof why);
    if (rc) return sfail(nullptr, rc, "%s", why);
    const Sizes s = sizes_of(cfg);
    if (!d_params || !d_ws || bytes < (size_t)s.total)
        return sfail(nullptr, SUR_ESIZE, "workspace of %zu bytes is smaller than the %lld needed", bytes, s.total);
    if (((uintptr_t)d_ws) & 255) return sfail(nullptr, SUR_EINVAL, "workspace must be 256-byte aligned");
    sur_net* n = (sur_net*)calloc(1, sizeof(sur_net));
    if (!n) return sfail(nullptr, SUR_EDEVICE, "out of host memory");
    n->cfg = *cfg;
    n->s = (hipStream_t)hip_stream;
    n->prm = d_params;
    n->oW0 = s.oW0; n->ob0 = s.ob0; n->oRr = s.oRr; n->oRi = s.oRi; n->oW = s.oW; n->ob = s.ob;
    n->oW1 = s.oW1; n->ob1 = s.ob1; n->oW2 = s.oW2; n->ob2 = s.ob2; n->n_params = s.n_params;
    float* w = (float*)d_ws;
    n->F = w + s.F; n->G = w + s.G; n->u = w + s.u; n->z = w + s.z; n->X = w + s.X; n->Y = w + s.Y;
    n->zh = w + s.zh; n->h = w + s.h; n->dA = w + s.dA; n->dB = w + s.dB; n->dX = w + s.dX; n->dY = w + s.dY;
    n->part = w + s.part; n->split = w + s.split; n->m1 = w + s.m1; n->m2 = w + s.m2;
    n->last_B = 0;
    const long long nm = (long long)cfg->n_points * cfg->modes;
    hipLaunchKernelGGL(k_dft_basis, dim3(nblk(nm, 256)), dim3(256), 0, n->s, n->F, n->G, cfg->n_points, cfg->modes);
    hipError_t e = hipMemsetAsync(n->m1, 0, (size_t)s.n_params * 4, n->s);
    if (e == hipSuccess) e = hipMemsetAsync(n->m2, 0, (size_t)s.n_params * 4, n->s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        free(n);
        return sfail(nullptr, SUR_EDEVICE, "init kernels failed: %s", hipGetErrorString(e));
    }
    *out = n;
    return SUR_OK;
}

int sur_forward(sur_net* n, int32_t B, const float* d_x, float* d_y)
{
    if (!n) return sfail(nullptr, SUR_EINVAL, "net is NULL");
    const sur_cfg& c = n->cfg;
    if (B < 1 || B > c.max_batch) return sfail(n, SUR_EINVAL, "batch %d outside 1..%d", B, c.max_batch);
    if (!d_x || !d_y) return sfail(n, SUR_EINVAL, "null input or output");
    const int Np = c.n_points, C = c.width, M2 = 2 * c.modes, P = c.proj;
    const long long Bn = (long long)B * Np, act = Bn * C, spec = (long long)B * M2 * C;
    const long long act_max = (long long)c.max_batch * Np * C, spec_max = (long long)c.max_batch * M2 * C;
    float* prm = n->prm;
    int rc = SUR_OK;
    // lift
    rc |= gemm(n->s, 0, 0, (int)Bn, C, c.c_in, 1.0f, d_x, c.c_in, 0, prm + n->oW0, C, 0, 0.0f, n->u, C, 0, 1, n->split);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(act, 256)), dim3(256), 0, n->s, n->u, prm + n->ob0, (float*)nullptr,
                       Bn, C, 0);
    for (int l = 0; l < c.layers; ++l) {
        float* ul = n->u + l * act_max;
        float* un = n->u + (l + 1) * act_max;
        float* X = n->X + l * spec_max;
        const float* Rr = prm + n->oRr + (long long)l * c.modes * C * C;
        const float* Ri = prm + n->oRi + (long long)l * c.modes * C * C;
        // X_b = F^T u_b
        rc |= gemm(n->s, 1, 0, M2, C, Np, 1.0f, n->F, M2, 0, ul, C, (long long)Np * C, 0.0f, X, C,
                   (long long)M2 * C, B, n->split);
        // per mode m: Yr = Xr Rr - Xi Ri, Yi = Xr Ri + Xi Rr (rows b, stride 2 modes x C)
        const int ldx = M2 * C;
        rc |= gemm(n->s, 0, 0, B, C, C, 1.0f, X, ldx, 2 * C, Rr, C, (long long)C * C, 0.0f, n->Y, ldx, 2 * C, c.modes, n->split);
        rc |= gemm(n->s, 0, 0, B, C, C, -1.0f, X + C, ldx, 2 * C, Ri, C, (long long)C * C, 1.0f, n->Y, ldx, 2 * C,
                   c.modes, n->split);
        rc |= gemm(n->s, 0, 0, B, C, C, 1.0f, X, ldx, 2 * C, Ri, C, (long long)C * C, 0.0f, n->Y + C, ldx, 2 * C,
                   c.modes, n->split);
        rc |= gemm(n->s, 0, 0, B, C, C, 1.0f, X + C, ldx, 2 * C, Rr, C, (long long)C * C, 1.0f, n->Y + C, ldx,
                   2 * C, c.modes, n->split);
        // z = G Y_b + u W + b
        rc |= gemm(n->s, 0, 0, Np, C, M2, 1.0f, n->G, M2, 0, n->Y, C, (long long)M2 * C, 0.0f, un, C,
                   (long long)Np * C, B, n->split);
        rc |= gemm(n->s, 0, 0, (int)Bn, C, C, 1.0f, ul, C, 0, prm + n->oW + (long long)l * C * C, C, 0, 1.0f, un, C,
                   0, 1, n->split);
        const int last = (l == c.layers - 1);
        hipLaunchKernelGGL(k_bias_act, dim3(nblk(act, 256)), dim3(256), 0, n->s, un, prm + n->ob + (long long)l * C,
                           n->z + l * act_max, Bn, C, last ? 0 : 1);
    }
    // projection
    float* uL = n->u + c.layers * act_max;
    rc |= gemm(n->s, 0, 0, (int)Bn, P, C, 1.0f, uL, C, 0, prm + n->oW1, P, 0, 0.0f, n->h, P, 0, 1, n->split);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(Bn * P, 256)), dim3(256), 0, n->s, n->h, prm + n->ob1, n->zh, Bn, P, 1);
    rc |= gemm(n->s, 0, 0, (int)Bn, c.c_out, P, 1.0f, n->h, P, 0, prm + n->oW2, c.c_out, 0, 0.0f, d_y, c.c_out, 0, 1, n->split);
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(Bn * c.c_out, 256)), dim3(256), 0, n->s, d_y, prm + n->ob2,
                       (float*)nullptr, Bn, c.c_out, 0);
    if (rc || hipGetLastError() != hipSuccess) return sfail(n, SUR_EDEVICE, "forward launch failed");
    n->last_B = B;
    (void)spec;
    return SUR_OK;
}

int sur_backward(sur_net* n, int32_t B, const float* d_x, const float* d_dy, float* d_grad)
{
    if (!n) return sfail(nullptr, SUR_EINVAL, "net is NULL");
    const sur_cfg& c = n->cfg;
    if (B != n->last_B) return sfail(n, SUR_ESTATE, "backward of batch %d needs a forward of that batch first", B);
    if (!d_x || !d_dy || !d_grad) return sfail(n, SUR_EINVAL, "null argument");
    const int Np = c.n_points, C = c.width, M2 = 2 * c.modes, P = c.proj;
    const long long Bn = (long long)B * Np, act = Bn * C;
    const long long act_max = (long long)c.max_batch * Np * C, spec_max = (long long)c.max_batch * M2 * C;
    const float* prm = n->prm;
    float* g = d_grad;
    int rc = SUR_OK;
    // projection: y = h W2 + b2, h = gelu(zh), zh = uL W1 + b1
    rc |= gemm(n->s, 1, 0, P, c.c_out, (int)Bn, 1.0f, n->h, P, 0, d_dy, c.c_out, 0, 0.0f, g + n->oW2, c.c_out, 0, 1, n->split);
    colsum(n, d_dy, Bn, c.c_out, g + n->ob2, 0.0f);
    float* dh = n->dA;
    rc |= gemm(n->s, 0, 1, (int)Bn, P, c.c_out, 1.0f, d_dy, c.c_out, 0, prm + n->oW2, c.c_out, 0, 0.0f, dh, P, 0, 1, n->split);
    hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk(Bn * P, 256)), dim3(256), 0, n->s, dh, n->zh, Bn * P);
    const float* uL = n->u + c.layers * act_max;
    rc |= gemm(n->s, 1, 0, C, P, (int)Bn, 1.0f, uL, C, 0, dh, P, 0, 0.0f, g + n->oW1, P, 0, 1, n->split);
    colsum(n, dh, Bn, P, g + n->ob1, 0.0f);
    float* du = n->dB;
    rc |= gemm(n->s, 0, 1, (int)Bn, C, P, 1.0f, dh, P, 0, prm + n->oW1, P, 0, 0.0f, du, C, 0, 1, n->split);
    // Fourier layers, last to first; du holds dL/du_{l+1} on entry
    for (int l = c.layers - 1; l >= 0; --l) {
        const float* ul = n->u + l * act_max;
        const float* X = n->X + l * spec_max;
        const float* Rr = prm + n->oRr + (long long)l * c.modes * C * C;
        const float* Ri = prm + n->oRi + (long long)l * c.modes * C * C;
        float* gRr = g + n->oRr + (long long)l * c.modes * C * C;
        float* gRi = g + n->oRi + (long long)l * c.modes * C * C;
        float* dz = du;
        if (l != c.layers - 1)
            hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk(act, 256)), dim3(256), 0, n->s, dz, n->z + l * act_max, act);
        colsum(n, dz, Bn, C, g + n->ob + (long long)l * C, 0.0f);
        rc |= gemm(n->s, 1, 0, C, C, (int)Bn, 1.0f, ul, C, 0, dz, C, 0, 0.0f, g + n->oW + (long long)l * C * C, C, 0, 1, n->split);
        // dY_b = G^T dz_b
        rc |= gemm(n->s, 1, 0, M2, C, Np, 1.0f, n->G, M2, 0, dz, C, (long long)Np * C, 0.0f, n->dY, C,
                   (long long)M2 * C, B, n->split);
        const int ldx = M2 * C;
        const float* dYr = n->dY;
        const float* dYi = n->dY + C;
        const float* Xr = X;
        const float* Xi = X + C;
        // dRr = Xr^T dYr + Xi^T dYi, dRi = Xr^T dYi - Xi^T dYr (per mode)
        rc |= gemm(n->s, 1, 0, C, C, B, 1.0f, Xr, ldx, 2 * C, dYr, ldx, 2 * C, 0.0f, gRr, C, (long long)C * C, c.modes, n->split);
        rc |= gemm(n->s, 1, 0, C, C, B, 1.0f, Xi, ldx, 2 * C, dYi, ldx, 2 * C, 1.0f, gRr, C, (long long)C * C, c.modes, n->split);
        rc |= gemm(n->s, 1, 0, C, C, B, 1.0f, Xr, ldx, 2 * C, dYi, ldx, 2 * C, 0.0f, gRi, C, (long long)C * C, c.modes, n->split);
        rc |= gemm(n->s, 1, 0, C, C, B, -1.0f, Xi, ldx, 2 * C, dYr, ldx, 2 * C, 1.0f, gRi, C, (long long)C * C, c.modes, n->split);
        // dXr = dYr Rr^T + dYi Ri^T, dXi = dYi Rr^T - dYr Ri^T
        rc |= gemm(n->s, 0, 1, B, C, C, 1.0f, dYr, ldx, 2 * C, Rr, C, (long long)C * C, 0.0f, n->dX, ldx, 2 * C, c.modes, n->split);
        rc |= gemm(n->s, 0, 1, B, C, C, 1.0f, dYi, ldx, 2 * C, Ri, C, (long long)C * C, 1.0f, n->dX, ldx, 2 * C, c.modes, n->split);
        rc |= gemm(n->s, 0, 1, B, C, C, 1.0f, dYi, ldx, 2 * C, Rr, C, (long long)C * C, 0.0f, n->dX + C, ldx, 2 * C,
                   c.modes, n->split);
        rc |= gemm(n->s, 0, 1, B, C, C, -1.0f, dYr, ldx, 2 * C, Ri, C, (long long)C * C, 1.0f, n->dX + C, ldx, 2 * C,
                   c.modes, n->split);
        // du_l = dz W^T + F dX_b  (into the other scratch, then swap)
        float* dn = (du == n->dB) ? n->dA : n->dB;
        rc |= gemm(n->s, 0, 1, (int)Bn, C, C, 1.0f, dz, C, 0, prm + n->oW + (long long)l * C * C, C, 0, 0.0f, dn, C, 0, 1, n->split);
        rc |= gemm(n->s, 0, 0, Np, C, M2, 1.0f, n->F, M2, 0, n->dX, C, (long long)M2 * C, 1.0f, dn, C,
                   (long long)Np * C, B, n->split);
        du = dn;
    }
    // lift: u0 = x W0 + b0
    rc |= gemm(n->s, 1, 0, c.c_in, C, (int)Bn, 1.0f, d_x, c.c_in, 0, du, C, 0, 0.0f, g + n->oW0, C, 0, 1, n->split);
    colsum(n, du, Bn, C, g + n->ob0, 0.0f);
    if (rc || hipGetLastError() != hipSuccess) return sfail(n, SUR_EDEVICE, "backward launch failed");
    return SUR_OK;
}

int sur_loss(sur_net* n, int32_t B, const float* d_y, const float* d_t, const float* d_mask, const float* d_wo,
             float* d_dy, float* d_loss)
{
    if (!n) return sfail(nullptr, SUR_EINVAL, "net is NULL");
    const sur_cfg& c = n->cfg;
    if (B < 1 || B > c.max_batch || !d_y || !d_t || !d_wo || !d_dy || !d_loss)
        return sfail(n, SUR_EINVAL, "bad loss arguments");
    const long long cnt = (long long)B * c.n_points * c.c_out;
    const unsigned nb = nblk(cnt, 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, n->s, d_y, d_t, d_mask, d_wo, cnt, c.c_out,
                       1.0f / (float)((long long)B * c.n_points), d_dy, n->part);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, n->s, n->part, (int)nb, d_loss);
    return hipGetLastError() == hipSuccess ? SUR_OK : sfail(n, SUR_EDEVICE, "loss launch failed");
}

int sur_adam(sur_net* n, const float* d_grad, float lr, float beta1, float beta2, float eps, int64_t step)
{
    if (!n || !d_grad || step < 1) return sfail(n, SUR_EINVAL, "bad Adam arguments");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n->n_params, 256)), dim3(256), 0, n->s, n->prm, d_grad, n->m1, n->m2,
                       n->n_params, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? SUR_OK : sfail(n, SUR_EDEVICE, "Adam launch failed");
}

int sur_reset_moments(sur_net* n)
{
    if (!n) return sfail(nullptr, SUR_EINVAL, "net is NULL");
    hipError_t e = hipMemsetAsync(n->m1, 0, (size_t)n->n_params * 4, n->s);
    if (e == hipSuccess) e = hipMemsetAsync(n->m2, 0, (size_t)n->n_params * 4, n->s);
    return e == hipSuccess ? SUR_OK : sfail(n, SUR_EDEVICE, "%s", hipGetErrorString(e));
}

int sur_gemm(int32_t transA, int32_t transB, int32_t M, int32_t N, int32_t K, float alpha, const float* A,
             int32_t lda, int64_t sA, const float* B, int32_t ldb, int64_t sB, float beta, float* C, int32_t ldc,
             int64_t sC, int32_t batch, void* hip_stream)
{
    if (M < 0 || N < 0 || K < 0 || batch < 0 || (transA != 0 && transA != 1) || (transB != 0 && transB != 1))
        return sfail(nullptr, SUR_EINVAL, "bad GEMM shape");
    if ((M && N && batch) && (!A || !B || !C)) return sfail(nullptr, SUR_EINVAL, "null matrix");
    if (lda < (transA ? M : K) || ldb < (transB ? K : N) || ldc < N)
        return sfail(nullptr, SUR_EINVAL, "leading dimension too small");
    int rc = gemm((hipStream_t)hip_stream, transA, transB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                  batch);
    return rc ? sfail(nullptr, rc, "GEMM launch failed") : SUR_OK;
}

int sur_destroy(sur_net* n)
{
    free(n);
    return SUR_OK;
}

const char* sur_last_error(const sur_net* n) { return n ? n->err : g_serr; }

}  // extern "C"
