/*
 * islbm_mlp.h -- C-ABI of the learned warm start's neural-network kernels
 * (gfx950, BF16 matrix cores with FP32 accumulation).
 *
 * The warm start predicts the steady velocity and temperature of the cavity
 * (2-D: u, v, T from x, y, log10 Ra; 3-D: u, v, w, T from x, y, z, log10 Ra)
 * at an unseen Rayleigh number from a coordinate network trained on fields the
 * solver produced; the prediction sets equilibrium initial populations
 * (islbm_init_fields_device), and the solver then runs as usual.  These entry
 * points are the building blocks of its training and inference: Fourier
 * features, one generic BF16 GEMM with fused epilogues, the loss gradient,
 * column sums, gathers and the Adam update.
 *
 * Conventions: matrices are row-major with explicit leading dimensions (in
 * elements); "bf16" buffers hold IEEE bfloat16 (2 bytes); all pointers are
 * device pointers owned by the caller; `stream` is a hipStream_t (NULL = the
 * default stream).  Work is enqueued asynchronously.  Every call returns 0,
 * or -1 (ISLBM_EINVAL) for a NULL pointer, a non-positive size or an unknown
 * mode, or -5 (ISLBM_EDEVICE) when the launch fails.
 */
#ifndef ISLBM_MLP_H
#define ISLBM_MLP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fourier features of p (n x 3 floats, ld 3): for f < F,
 * out[i][f] = sin(2 pi <B_f, p_i>), out[i][F + f] = cos(2 pi <B_f, p_i>),
 * B is F x 3 floats.  out: bf16, n x (2F), leading dimension ldo. */
int islbm_mlp_features(const float* p, int n, const float* B, int F, void* out, int ldo,
                       void* stream);

/* The same for d inputs per point (1 <= d <= 8): p is n x d floats (ld d), B is
 * F x d floats; out[i][f] = sin(2 pi <B_f, p_i>), out[i][F + f] = cos(...).
 * The 3-D cavity uses d = 4 (x, y, z, log10 Ra - 7). */
int islbm_mlp_features_d(const float* p, int n, int d, const float* B, int F, void* out, int ldo,
                         void* stream);

/* GEMM modes (A, B bf16; accumulation FP32 on the matrix cores):
 *   0 (NT): C[M][N] = sum_k A[m][k] B[n][k]    (A: M x K, B: N x K)
 *   1 (NN): C[M][N] = sum_k A[m][k] B[k][n]    (A: M x K, B: K x N)
 *   2 (TN): C[M][N] = sum_k A[k][m] B[k][n]    (A: K x M, B: K x N); split over K
 *           into workspace partials (FP32, needs >= 4*M*N*ceil(K/1024) bytes,
 *           NULL => one split), then summed in a fixed order.
 * Epilogues (bias has N floats, aux is M x N floats with leading dim ldaux):
 *   0: C = acc (FP32)
 *   1: C = acc + bias (FP32 pre-activation); Cb = bf16(silu(C))
 *   2: C = acc + bias
 *   3: C = acc * silu'(aux) (FP32); Cb = bf16(C)            [backward through SiLU]
 * C (FP32, ldc) and Cb (bf16, ldcb) may be NULL when not needed by the epilogue. */
int islbm_gemm_bf16(int mode, int M, int N, int K, const void* A, int lda, const void* B,
                    int ldb, float* C, int ldc, void* Cb, int ldcb, const float* bias,
                    const float* aux, int ldaux, int epilogue, float* workspace,
                    size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the TN
 * product of islbm_gemm_bf16 (mode 2, epilogue 0: C[M][N] = sum_k A[k][m] B[k][n],
 * A: K x M bf16 with leading dimension lda >= M, B: K x N bf16 with ldb >= N,
 * C: M x N floats with ldc >= N), its split-K partials held in a fixed 8 MiB
 * device array inside the library instead of a workspace argument; the
 * result equals that of islbm_gemm_bf16 with a workspace, bit for bit.  It
 * allocates nothing (the array's device address is looked up once per device
 * on the first call).  Limit: 4 * M * N * ceil(K / 1024) bytes <= 8 MiB, else
 * -1 (ISLBM_EINVAL) with nothing launched; -1 also for NULL pointers or
 * non-positive sizes, -5 for a launch or symbol-lookup failure.  All calls on
 * one GPU share that array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller. */
int islbm_gemm_bf16_tn_noalloc(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                               float* C, int ldc, void* stream);

/* Weighted mean-squared-error gradient: for i < n, j < m,
 * r = y[i][j] - t[i][j]; g[i][j] = 2 w_j r / n (FP32 into gf and bf16 into gb,
 * either may be NULL); loss_out[0] = sum_ij w_j r^2 / n (FP64, one value,
 * written by a fixed-order reduction). */
int islbm_mlp_mse_grad(const float* y, int ldy, const float* t, int ldt, const float* w, int n,
                       int m, float* gf, void* gb, int ldg, double* loss_out, void* stream);

/* Column sums of an n x m FP32 matrix (fixed-order reduction): out[j] = sum_i a[i][j]. */
int islbm_mlp_colsum(const float* a, int n, int m, int lda, float* out, void* stream);

/* Row gather: dst[i][:] = src[idx[i]][:] for i < n (floats, width cols). */
int islbm_mlp_gather(const float* src, int lds, const int* idx, int n, int cols, float* dst,
                     int ldd, void* stream);

/* FP32 -> bf16 conversion of count values (round to nearest even). */
int islbm_f32_to_bf16(const float* src, void* dst, size_t count, void* stream);

/* Adam step with decoupled weight decay on count FP32 parameters:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + wd w); wb = bf16(w) (optional). */
int islbm_mlp_adam(float* w, const float* g, float* m, float* v, void* wb, size_t count,
                   float lr, float b1, float b2, float eps, float wd, int t, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ISLBM_MLP_H */
