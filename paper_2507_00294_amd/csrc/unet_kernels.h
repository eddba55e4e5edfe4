// unet_kernels.h -- launchers of the surrogate's HIP kernels (unet_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dd {
namespace nn {

// C = A B on BF16 MFMA (FP32 accumulation); ta/tb select transposed storage
// (see k_gemm); with ksplit > 1, gemm_splits() partial matrices are written at
// C + s*M*ldc and must be added by sum_splits.
hipError_t gemm(const __bf16* A, int lda, bool ta, const __bf16* B, int ldb, bool tb, float* C,
                int ldc, int M, int N, int K, int ksplit, hipStream_t st);
int gemm_splits(int M, int K, int ksplit);
// act = SiLU(A B + bias), z = A B + bias.
hipError_t gemm_bias_silu(const __bf16* A, int lda, const __bf16* B, int ldb, float* act, float* z,
                          int ldc, const float* bias, int M, int N, int K, hipStream_t st);
hipError_t sum_splits(const float* part, int splits, int64_t n, float* out, hipStream_t st);
hipError_t im2col(const float* x, int B, int H, int W, int C, __bf16* col, hipStream_t st);
hipError_t col2im(const float* dcol, int B, int H, int W, int C, float* dx, hipStream_t st);
hipError_t silu_bwd(const float* dA, const float* Z, int64_t n, float* dZ, __bf16* dZb,
                    hipStream_t st);
hipError_t colsum_add(const float* dZ, int M, int N, float* db, hipStream_t st);
hipError_t pool_fwd(const float* x, int B, int H, int W, int C, float* y, hipStream_t st);
hipError_t pool_bwd_add(const float* dy, int B, int H, int W, int C, float* dx, hipStream_t st);
hipError_t up_concat(const float* x, int B, int h, int w, int C1, const float* skip, int C2,
                     float* out, hipStream_t st);
hipError_t up_concat_bwd(const float* dout, int B, int h, int w, int C1, int C2, float* dx,
                         float* dskip, hipStream_t st);
hipError_t head_fwd(const float* a, int64_t M, int C, const float* w, const float* b, float* y,
                    hipStream_t st);
hipError_t head_bwd(const float* dy, const float* a, int64_t M, int C, const float* w, float* da,
                    float* dw, hipStream_t st);
hipError_t mse(const float* y, const float* t, int64_t n, float* dy, double* partial, int nblocks,
               hipStream_t st);
hipError_t adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                float eps, float bc1, float bc2, __bf16* wb, hipStream_t st);
hipError_t to_bf16(const float* x, int64_t n, __bf16* y, hipStream_t st);
hipError_t fill(float* x, int64_t n, float v, hipStream_t st);
hipError_t exp_out(const float* y, int64_t n, int64_t per_map, const double* pref, double* psi,
                   hipStream_t st);
hipError_t log_target(const double* psi, int64_t n, int64_t per_map, const double* pref, float* t,
                      hipStream_t st);

}  // namespace nn
}  // namespace dd
