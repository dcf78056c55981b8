/*
 * surrogate.h -- C ABI of the learned surrogate of the FDTD march: a
 * one-dimensional Fourier neural operator trained on the solver's outputs
 * (P_e(t) on a fixed time grid and the two-photon amplitude chi of Eq. (2) at
 * the detectors), whose forward and backward passes run on bf16 matrix cores
 * with fp32 accumulation.  It is not part of the paper: the paper's method
 * is the march (fdtd.h), which also judges the surrogate's answers.
 *
 * Network, for inputs x of shape (B, n_points, c_in), row-major:
 *   u0 = x W0 + b0
 *   layer l < layers:  z_l = IDFT(R_l . DFT(u_l)) + u_l W_l + b_l,
 *                      u_{l+1} = gelu(z_l) (no activation after the last layer)
 *     DFT keeps the first `modes` Fourier modes of each channel; R_l holds one
 *     complex width x width matrix per mode (real parts Rr, imaginary Ri);
 *     IDFT is the inverse transform of a real signal with those modes only.
 *   y = gelu(u_L W1 + b1) W2 + b2, shape (B, n_points, c_out).
 * gelu(v) = v (1 + erf(v / sqrt 2)) / 2.
 *
 * Parameters: one fp32 device array of sur_sizes()'s n_params values, owned by
 * the caller, in this order (each row-major): W0 (c_in x width), b0 (width),
 * Rr (layers x modes x width x width), Ri (same), W (layers x width x width),
 * b (layers x width), W1 (width x proj), b1 (proj), W2 (proj x c_out),
 * b2 (c_out).  Row i of a weight matrix multiplies input channel i.
 *
 * Every matrix product reads fp32 operands, rounds them to bf16 and
 * accumulates in fp32; element-wise work is fp32.  All calls enqueue on the
 * stream given to sur_init and return without waiting.  Errors: SUR_OK or a
 * negative code, text from sur_last_error.
 */
#ifndef SURROGATE_H
#define SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sur_status {
    SUR_OK = 0,
    SUR_EINVAL = -1,    /* bad configuration or argument */
    SUR_ESIZE = -2,     /* workspace too small */
    SUR_ESTATE = -3,    /* backward without a forward of the same batch */
    SUR_EDEVICE = -4    /* HIP error */
};

typedef struct sur_cfg {
    uint32_t struct_size;   /* sizeof(sur_cfg) */
    int32_t n_points;       /* grid points per sample (>= 2) */
    int32_t c_in;           /* input channels */
    int32_t width;          /* channels of the Fourier layers */
    int32_t modes;          /* Fourier modes kept (<= n_points / 2) */
    int32_t layers;         /* Fourier layers */
    int32_t proj;           /* hidden channels of the projection */
    int32_t c_out;          /* output channels */
    int32_t max_batch;      /* largest batch a call may pass */
} sur_cfg;

typedef struct sur_net sur_net;

/* Parameter count and device workspace bytes (activations kept for the
 * backward pass, DFT bases, gradient scratch, Adam moments). */
int sur_sizes(const sur_cfg *cfg, int64_t *n_params, size_t *ws_bytes);

/* Bind parameters (device, fp32, n_params) and workspace (device, 256-byte
 * aligned, >= ws_bytes, caller-owned) on a HIP stream; builds the DFT bases
 * and clears the Adam moments. */
int sur_init(const sur_cfg *cfg, float *d_params, void *d_workspace, size_t bytes, void *hip_stream,
             sur_net **out);

/* y = net(x) for a batch of B <= max_batch samples (device pointers; x is
 * (B, n_points, c_in), y is (B, n_points, c_out)).  Keeps the activations for
 * sur_backward. */
int sur_forward(sur_net *net, int32_t B, const float *d_x, float *d_y);

/* Gradient of a scalar loss with respect to every parameter, given
 * dloss/dy (B, n_points, c_out) for the last sur_forward (same B and x);
 * writes n_params fp32 values to d_grad (overwritten, same order as the
 * parameters). */
int sur_backward(sur_net *net, int32_t B, const float *d_x, const float *d_dy, float *d_grad);

/* Masked, channel-weighted mean squared error:
 *   loss = sum_{b,p,o} wo[o] mask[b,p,o] (y - t)^2 / (B n_points)
 * and dy = dloss/dy.  mask may be NULL (all ones); wo has c_out values. */
int sur_loss(sur_net *net, int32_t B, const float *d_y, const float *d_t, const float *d_mask, const float *d_wo,
             float *d_dy, float *d_loss);

/* One Adam step on the parameters (bias-corrected moments; step counts from
 * 1). */
int sur_adam(sur_net *net, const float *d_grad, float lr, float beta1, float beta2, float eps, int64_t step);
int sur_reset_moments(sur_net *net);

/* The library's matrix product, for tests and callers: for z < batch,
 * C_z = alpha op(A_z) op(B_z) + beta C_z with op(A) M x K, op(B) K x N, all
 * row-major fp32 with leading dimensions lda, ldb, ldc and batch strides sA,
 * sB, sC (elements); trans = 1 means the stored matrix is the transpose.
 * Operands are rounded to bf16, accumulation is fp32. */
int sur_gemm(int32_t transA, int32_t transB, int32_t M, int32_t N, int32_t K, float alpha, const float *A,
             int32_t lda, int64_t sA, const float *B, int32_t ldb, int64_t sB, float beta, float *C, int32_t ldc,
             int64_t sC, int32_t batch, void *hip_stream);

/* The sweep's arithmetic around the network (any stream; enqueued).
 * sur_encode: the network's input for B instances, (B, n, 8) float32 into
 *   d_x: the incident packet phi(-a - sigma) at sigma_p = 16 w p/(n-1)
 *   without its normalisation (real, imaginary), then Gamma 2a / 10,
 *   k0 a / 2 pi, ln w / ln 5, Delta / 0.01, ln(Gamma T) / ln 1000 and p/(n-1);
 *   d_par holds (w, k0, a, Gamma, Delta, T) per instance (B x 6 doubles), T
 *   the end of the P_e window.
 * sur_check: the a-posteriori check of a network's P_e (d_S) for B points of
 *   n samples, against FP64 solves of the same window and box on grids
 *   about 2x, 4x and 8x coarser (d_P2, d_P4, d_P8, each B x n), with grid
 *   steps (h_fine, h_2, h_4, h_8) per point in d_h (B x 4) and d_valid[b] = 0
 *   where a coarse grid does not exist.  The scheme is second order, so in
 *   its asymptotic range P_h = P + K h^2: the fine solve differs from P2 by
 *   about (P4 - P2)(h_2^2 - h_fine^2)/(h_4^2 - h_2^2), and the differences
 *   of successive coarse solves stand in the ratio
 *   rho = (h_8^2 - h_4^2)/(h_4^2 - h_2^2).  Per point (L2 norms over the
 *   samples): dist = |S - P2|/|P2|; est = safety |P4 - P2|/|P2| times that
 *   factor; q = (|P8 - P4|/|P4 - P2|)/rho, which is 1 in the asymptotic
 *   range.  The point is in range when |q - 1| <= ratio_tol; it is accepted
 *   for the coarse solve alone when in range and est <= tol, for the network
 *   when in range and dist + est <= tol (so every point accepted for the
 *   network is accepted for the coarse solve).  Writes (dist, est, q) into
 *   d_out (B x 3 doubles) and the two decisions into d_acc (B x 2 int32).
 * Both return SUR_EINVAL for null pointers or sizes out of range (n >= 2 for
 * sur_encode, n >= 1 for sur_check, B >= 0; B = 0 enqueues nothing). */
int sur_encode(const double *d_par, int32_t B, int32_t n, float *d_x, void *hip_stream);
int sur_check(const double *d_S, const double *d_P2, const double *d_P4, const double *d_P8, const double *d_h,
              const int32_t *d_valid, int32_t B, int32_t n, double tol, double safety, double ratio_tol,
              double *d_out, int32_t *d_acc, void *hip_stream);

int sur_destroy(sur_net *net);
const char *sur_last_error(const sur_net *net);

#ifdef __cplusplus
}
#endif

#endif /* SURROGATE_H */
