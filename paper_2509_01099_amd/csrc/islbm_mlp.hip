// Neural-network kernels of the learned warm start (gfx950): Fourier
// features, a BF16 matrix-core GEMM with FP32 accumulation and fused
// epilogues, the MSE gradient, column sums, gathers and Adam.
//
// The GEMM uses v_mfma_f32_32x32x16_bf16: a 256-thread workgroup computes a
// 64 x 64 tile of C as four 32 x 32 wave tiles, stepping through K in slices
// of 32 staged in LDS in a K-contiguous layout (so the three operand layouts
// of the forward pass, the data gradient and the weight gradient share the
// same inner loop and differ only in how a slice is loaded).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <mutex>

#include "../../include/islbm_mlp.h"

namespace islbm_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;  // LDS rows padded by 16 bytes
constexpr int KSPLIT = 1024;                            // K per split of the TN mode

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ __bf16 ld_bf(const __bf16* p) { return *p; }

// Staging of one BK-slice of an operand into a [64][LDK] LDS tile, rows r0..
// r0+63 of `rows` and columns k0..k0+BK-1 (below kend).  Each thread moves 8
// consecutive elements with one 16-byte load when they lie inside the
// operand and the address is 16-byte aligned, else element by element (edges,
// odd leading dimensions); elements outside the operand are zero.
//   stage_k: the operand is rows x K with K contiguous (row r at src + r*ld);
//            a thread covers k..k+7 of one row, stored as one 16-byte row
//            segment of the tile.
//   stage_t: the operand is K x rows with rows contiguous (k at src + k*ld);
//            a thread covers rows r..r+7 of one k, stored transposed.
__device__ __forceinline__ void stage_k(const __bf16* __restrict__ src, int ld, int rows, int r0, int k0,
                                        int kend, __bf16 (*dst)[LDK]) {
  static_assert(BM == 64 && BN == 64 && BK == 32, "one 8-element unit per thread");
  const int r = threadIdx.x >> 2, kk = (threadIdx.x & 3) * 8;
  const int gr = r0 + r, gk = k0 + kk;
  const __bf16* p = src + (long long)gr * ld + gk;
  if (gr < rows && gk + 8 <= kend && (reinterpret_cast<size_t>(p) & 15) == 0) {
    *reinterpret_cast<bf16x8*>(&dst[r][kk]) = *reinterpret_cast<const bf16x8*>(p);
  } else {
    const __bf16 zero = __bf16(0.0f);
#pragma unroll
    for (int i = 0; i < 8; ++i) dst[r][kk + i] = (gr < rows && gk + i < kend) ? ld_bf(p + i) : zero;
  }
}

__device__ __forceinline__ void stage_t(const __bf16* __restrict__ src, int ld, int rows, int r0, int k0,
                                        int kend, __bf16 (*dst)[LDK]) {
  const int kk = threadIdx.x >> 3, r = (threadIdx.x & 7) * 8;
  const int gk = k0 + kk, gr = r0 + r;
  const __bf16* p = src + (long long)gk * ld + gr;
  if (gk < kend && gr + 8 <= rows && (reinterpret_cast<size_t>(p) & 15) == 0) {
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(p);
#pragma unroll
    for (int i = 0; i < 8; ++i) dst[r + i][kk] = v[i];
  } else {
    const __bf16 zero = __bf16(0.0f);
#pragma unroll
    for (int i = 0; i < 8; ++i) dst[r + i][kk] = (gk < kend && gr + i < rows) ? ld_bf(p + i) : zero;
  }
}

template <int MODE, int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                                   const __bf16* __restrict__ B, int ldb, float* __restrict__ C,
                                                   int ldc, __bf16* __restrict__ Cb, int ldcb,
                                                   const float* __restrict__ bias, const float* __restrict__ aux,
                                                   int ldaux, float* __restrict__ ws, int kchunk) {
  __shared__ __attribute__((aligned(16))) __bf16 As[BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][LDK];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // A slice -> As[m][k], B slice -> Bs[n][k]
    if constexpr (MODE == 2) stage_t(A, lda, M, m0, k0, kend, As);  // A is K x M (M contiguous)
    else stage_k(A, lda, M, m0, k0, kend, As);                      // A is M x K (K contiguous)
    if constexpr (MODE == 0) stage_k(B, ldb, N, n0, k0, kend, Bs);  // B is N x K (K contiguous)
    else stage_t(B, ldb, N, n0, k0, kend, Bs);                      // B is K x N (N contiguous)
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm + (lane & 31)][kk + 8 * (lane >> 5)]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn + (lane & 31)][kk + 8 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  // accumulator i of lane l holds C[8(i/4) + 4(l/32) + i%4][l%32] of the wave tile
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    if (m >= M || n >= N) continue;
    float v = acc[i];
    if constexpr (MODE == 2) {
      ws[((long long)blockIdx.z * M + m) * N + n] = v;
    } else if constexpr (EPI == 0) {
      C[(long long)m * ldc + n] = v;
    } else if constexpr (EPI == 1) {
      v += bias[n];
      if (C) C[(long long)m * ldc + n] = v;
      Cb[(long long)m * ldcb + n] = __bf16(silu(v));
    } else if constexpr (EPI == 2) {
      C[(long long)m * ldc + n] = v + bias[n];
    } else {
      v *= dsilu(aux[(long long)m * ldaux + n]);
      if (C) C[(long long)m * ldc + n] = v;
      if (Cb) Cb[(long long)m * ldcb + n] = __bf16(v);
    }
  }
}

// Fixed-order sum of the split-K partials of the TN mode.
__global__ void splitk_sum_kernel(const float* __restrict__ ws, int splits, int M, int N, float* __restrict__ C,
                                  int ldc) {
  const long long total = (long long)M * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += ws[z * total + e];
    C[(e / N) * ldc + (e % N)] = s;
  }
}

__global__ void features_kernel(const float* __restrict__ p, int n, int d, const float* __restrict__ B, int F,
                                __bf16* __restrict__ out, int ldo) {
  const long long total = (long long)n * F;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / F;
    const int f = (int)(e % F);
    float dot = 0.0f;
    for (int c = 0; c < d; ++c) dot += B[(long long)d * f + c] * p[(long long)d * i + c];
    const float z = 6.283185307179586f * dot;
    out[i * ldo + f] = __bf16(sinf(z));
    out[i * ldo + F + f] = __bf16(cosf(z));
  }
}

__global__ void __launch_bounds__(1024) mse_grad_kernel(const float* __restrict__ y, int ldy,
                                                        const float* __restrict__ t, int ldt,
                                                        const float* __restrict__ w, int n, int m,
                                                        float* __restrict__ gf, __bf16* __restrict__ gb, int ldg,
                                                        double* __restrict__ loss_out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  const long long total = (long long)n * m;
  for (long long e = threadIdx.x; e < total; e += blockDim.x) {
    const long long i = e / m;
    const int j = (int)(e % m);
    const float r = y[i * ldy + j] - t[i * ldt + j];
    const float g = 2.0f * w[j] * r / float(n);
    if (gf) gf[i * ldg + j] = g;
    if (gb) gb[i * ldg + j] = __bf16(g);
    acc += double(w[j]) * double(r) * double(r);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_out) loss_out[0] = sh[0] / double(n);
}

__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ a, int n, int m, int lda,
                                                     float* __restrict__ out) {
  __shared__ float sh[256];
  const int j = blockIdx.x;
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += a[(long long)i * lda + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sh[0];
}

__global__ void gather_kernel(const float* __restrict__ src, int lds, const int* __restrict__ idx, int n, int cols,
                              float* __restrict__ dst, int ldd) {
  const long long total = (long long)n * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / cols;
    const int c = (int)(e % cols);
    dst[i * ldd + c] = src[(long long)idx[i] * lds + c];
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ src, __bf16* __restrict__ dst, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = __bf16(src[e]);
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, __bf16* __restrict__ wb, size_t count, float lr, float b1,
                            float b2, float eps, float wd, float c1, float c2) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[e]);
    w[e] = wi;
    if (wb) wb[e] = __bf16(wi);
  }
}

static int grid_for(long long total) {
  long long b = (total + 255) / 256;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

static int status(hipError_t e) { return e == hipSuccess ? 0 : -5; }

template <int MODE, int EPI>
static hipError_t gemm_launch(int M, int N, int K, const void* A, int lda, const void* B, int ldb, float* C, int ldc,
                              void* Cb, int ldcb, const float* bias, const float* aux, int ldaux, float* ws,
                              int splits, int kchunk, hipStream_t st) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, splits);
  hipLaunchKernelGGL((gemm_kernel<MODE, EPI>), grid, dim3(256), 0, st, M, N, K, static_cast<const __bf16*>(A), lda,
                     static_cast<const __bf16*>(B), ldb, C, ldc, static_cast<__bf16*>(Cb), ldcb, bias, aux, ldaux,
                     ws, kchunk);
  return hipGetLastError();
}

}  // namespace islbm_mlp

using namespace islbm_mlp;

// ---------------------------------------------------------------------------
// Allocation-free TN product: the split-K partials live in a file-scope device
// array instead of a caller workspace.  Host code never passes the array's
// name to a kernel: it takes the array's device address once per device with
// hipGetSymbolAddress and passes that.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;  // 8 MiB per device
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

static std::once_flag g_scratch_once[kMaxDevices];
static float* g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];

// Device address of `scratch` on the current device (set up on the first call
// per device), or nullptr on failure.
static float* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? static_cast<float*>(ptr) : nullptr;
  });
  return g_scratch_ptr[dev];
}

extern "C" int islbm_gemm_bf16_tn_noalloc(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                                          float* C, int ldc, void* stream) {
  if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0 || lda < M || ldb < N || ldc < N) return -1;
  const int splits = (K + KSPLIT - 1) / KSPLIT;
  if ((size_t)4 * M * N * splits > kNoAllocScratchBytes) return -1;  // beyond the fixed scratch
  float* ws = scratch_on_current_device();
  if (!ws) return -5;
  hipStream_t st = (hipStream_t)stream;
  // every split writes its whole M x N slice before the fixed-order sum reads
  // it, so nothing of an earlier call's contents is read
  hipError_t e = gemm_launch<2, 0>(M, N, K, A, lda, B, ldb, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, ws, splits,
                                   KSPLIT, st);
  if (e != hipSuccess) return -5;
  hipLaunchKernelGGL(splitk_sum_kernel, dim3(grid_for((long long)M * N)), dim3(256), 0, st, ws, splits, M, N, C, ldc);
  return status(hipGetLastError());
}

extern "C" int islbm_mlp_features_d(const float* p, int n, int d, const float* B, int F, void* out, int ldo,
                                    void* stream) {
  if (!p || !B || !out || n <= 0 || d <= 0 || d > 8 || F <= 0 || ldo < 2 * F) return -1;
  hipLaunchKernelGGL(features_kernel, dim3(grid_for((long long)n * F)), dim3(256), 0, (hipStream_t)stream, p, n, d,
                     B, F, static_cast<__bf16*>(out), ldo);
  return status(hipGetLastError());
}

extern "C" int islbm_mlp_features(const float* p, int n, const float* B, int F, void* out, int ldo, void* stream) {
  return islbm_mlp_features_d(p, n, 3, B, F, out, ldo, stream);
}

extern "C" int islbm_gemm_bf16(int mode, int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                               float* C, int ldc, void* Cb, int ldcb, const float* bias, const float* aux, int ldaux,
                               int epilogue, float* workspace, size_t workspace_bytes, void* stream) {
  if (!A || !B || M <= 0 || N <= 0 || K <= 0 || mode < 0 || mode > 2 || epilogue < 0 || epilogue > 3) return -1;
  if ((epilogue == 0 || epilogue == 2) && !C) return -1;
  if (epilogue == 1 && !Cb) return -1;
  if ((epilogue == 1 || epilogue == 2) && !bias) return -1;
  if (epilogue == 3 && (!aux || (!C && !Cb))) return -1;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (mode == 2) {
    if (epilogue != 0 || !C) return -1;
    const int splits = (K + KSPLIT - 1) / KSPLIT;
    const size_t need = (size_t)4 * M * N * splits;
    if (workspace && workspace_bytes >= need) {
      // split K into independent slices, then a fixed-order sum of the slices
      e = gemm_launch<2, 0>(M, N, K, A, lda, B, ldb, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, workspace, splits,
                            KSPLIT, st);
      if (e != hipSuccess) return -5;
      hipLaunchKernelGGL(splitk_sum_kernel, dim3(grid_for((long long)M * N)), dim3(256), 0, st, workspace, splits, M,
                         N, C, ldc);
      return status(hipGetLastError());
    }
    // no workspace: one slice written straight into a dense M x N block of C
    if (ldc != N) return -1;
    return status(gemm_launch<2, 0>(M, N, K, A, lda, B, ldb, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, C, 1, K, st));
  }
#define GEMM_CASE(MD, EP)                                                                                       \
  if (mode == MD && epilogue == EP)                                                                             \
    return status(gemm_launch<MD, EP>(M, N, K, A, lda, B, ldb, C, ldc, Cb, ldcb, bias, aux, ldaux, nullptr, 1, \
                                      K, st));
  GEMM_CASE(0, 0)
  GEMM_CASE(0, 1)
  GEMM_CASE(0, 2)
  GEMM_CASE(0, 3)
  GEMM_CASE(1, 0)
  GEMM_CASE(1, 1)
  GEMM_CASE(1, 2)
  GEMM_CASE(1, 3)
#undef GEMM_CASE
  return -1;
}

extern "C" int islbm_mlp_mse_grad(const float* y, int ldy, const float* t, int ldt, const float* w, int n, int m,
                                  float* gf, void* gb, int ldg, double* loss_out, void* stream) {
  if (!y || !t || !w || n <= 0 || m <= 0) return -1;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, y, ldy, t, ldt, w, n, m, gf,
                     static_cast<__bf16*>(gb), ldg, loss_out);
  return status(hipGetLastError());
}

extern "C" int islbm_mlp_colsum(const float* a, int n, int m, int lda, float* out, void* stream) {
  if (!a || !out || n <= 0 || m <= 0) return -1;
  hipLaunchKernelGGL(colsum_kernel, dim3(m), dim3(256), 0, (hipStream_t)stream, a, n, m, lda, out);
  return status(hipGetLastError());
}

extern "C" int islbm_mlp_gather(const float* src, int lds, const int* idx, int n, int cols, float* dst, int ldd,
                                void* stream) {
  if (!src || !idx || !dst || n <= 0 || cols <= 0) return -1;
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for((long long)n * cols)), dim3(256), 0, (hipStream_t)stream, src, lds,
                     idx, n, cols, dst, ldd);
  return status(hipGetLastError());
}

extern "C" int islbm_f32_to_bf16(const float* src, void* dst, size_t count, void* stream) {
  if (!src || !dst || count == 0) return -1;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for((long long)count)), dim3(256), 0, (hipStream_t)stream, src,
                     static_cast<__bf16*>(dst), count);
  return status(hipGetLastError());
}

extern "C" int islbm_mlp_adam(float* w, const float* g, float* m, float* v, void* wb, size_t count, float lr, float b1,
                              float b2, float eps, float wd, int t, void* stream) {
  if (!w || !g || !m || !v || count == 0 || t <= 0) return -1;
  // bias corrections formed in double: 1 - b2^t loses most of its float
  // digits to cancellation when b2 is close to 1
  const float c1 = float(1.0 - pow((double)b1, (double)t)), c2 = float(1.0 - pow((double)b2, (double)t));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for((long long)count)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                     static_cast<__bf16*>(wb), count, lr, b1, b2, eps, wd, c1, c2);
  return status(hipGetLastError());
}
