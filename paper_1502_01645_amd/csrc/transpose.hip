// FP32 matrix transpose, the data movement of the alternating NNLS update of a nonnegative
// matrix factorisation (the use of NNLS the Introduction motivates): the W half of the update is
// an NNLS problem whose matrix and right-hand sides are H^T and V^T.
//
// 64 x 64 tiles through LDS (one column of padding against bank conflicts): 256 threads read a
// tile row-major with consecutive threads on consecutive columns and write it back with
// consecutive threads on consecutive rows of the source, so both global accesses are coalesced.
#include "../../include/nnls.h"
#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int TR_T = 64;

__global__ __launch_bounds__(256) void transpose_kernel(int64_t rows, int64_t cols,
                                                        const float* __restrict__ src,
                                                        int64_t ld_src, float* __restrict__ dst,
                                                        int64_t ld_dst) {
  __shared__ float t[TR_T][TR_T + 1];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * TR_T, c0 = (int64_t)blockIdx.x * TR_T;
#pragma unroll
  for (int u = 0; u < TR_T / 4; ++u) {
    const int rr = ty + 4 * u;
    const int64_t r = r0 + rr, c = c0 + tx;
    if (r < rows && c < cols) t[rr][tx] = src[r * ld_src + c];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < TR_T / 4; ++u) {
    const int cc = ty + 4 * u;
    const int64_t c = c0 + cc, r = r0 + tx;
    if (r < rows && c < cols) dst[c * ld_dst + r] = t[tx][cc];
  }
}

}  // namespace nnls

extern "C" int nnls_transpose(int64_t rows, int64_t cols, const float* src, int64_t ld_src,
                              float* dst, int64_t ld_dst, void* stream) {
  if (rows < 1 || cols < 1 || !src || !dst || ld_src < cols || ld_dst < rows) return NNLS_E_ARG;
  const int64_t gy = (rows + nnls::TR_T - 1) / nnls::TR_T;
  const int64_t gx = (cols + nnls::TR_T - 1) / nnls::TR_T;
  if (gy > 65535 || gx > (int64_t(1) << 31) - 1) return NNLS_E_UNSUPPORTED;
  hipLaunchKernelGGL(nnls::transpose_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0,
                     (hipStream_t)stream, rows, cols, src, ld_src, dst, ld_dst);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

namespace nnls {

// Y0[i, c] = s[i] * X[i, c]: a start point in the original variables mapped to the rescaled ones
// (rescaling (4), y = D^(1/2) x), the form in which Algorithm 2 takes a start.
__global__ __launch_bounds__(256) void rescale_start_kernel(int64_t n, int64_t k,
                                                            const double* __restrict__ s,
                                                            const float* __restrict__ X,
                                                            float* __restrict__ Y0) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * k) return;
  Y0[e] = (float)(s[e / k] * (double)X[e]);
}

}  // namespace nnls

extern "C" int nnls_rescale_start(int64_t n, int64_t k, const double* s, const float* X,
                                  float* Y0, void* stream) {
  if (n < 1 || k < 1 || !s || !X || !Y0) return NNLS_E_ARG;
  const int64_t blocks = (n * k + 255) / 256;
  if (blocks > (int64_t(1) << 31) - 1) return NNLS_E_UNSUPPORTED;
  hipLaunchKernelGGL(nnls::rescale_start_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)stream, n, k, s, X, Y0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}
