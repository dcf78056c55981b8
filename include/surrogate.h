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

int sur_destroy(sur_net *net);
const char *sur_last_error(const sur_net *net);

#ifdef __cplusplus
}
#endif

#endif /* SURROGATE_H */
