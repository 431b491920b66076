// Algorithm 2 with one workgroup per right-hand side (small and medium n, FP64 problems); the
// device code is in solve_core.hpp.  A single large right-hand side uses the whole-GPU solver
// and many FP32 right-hand sides the matrix-core solver instead.
#include "solve_core.hpp"

namespace nnls {

// Shared-Q form: column c of q / Y0 / X (leading dimension k).
template <typename T>
__global__ __launch_bounds__(SW_NT) void solve_wg_kernel(int64_t n, int64_t k, const T* Q,
                                                         const T* q, const double* s, double tol,
                                                         int max_iter, const T* Y0, T* X,
                                                         int32_t* iters, double* kkt,
                                                         int32_t* status, int64_t* rows_read,
                                                         float* trace, int trace_len, T* ws) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int64_t c = blockIdx.x;
  const SwLdsLayout L = sw_lds_layout(n, sizeof(T), SW_NT);
  T* lds_val = (T*)(smem + L.val);
  T* lds_val2 = (T*)(smem + L.val2);
  int* lds_idx = (int*)(smem + L.idx);
  int* lds_idx2 = (int*)(smem + L.idx2);
  T* redT = (T*)(smem + L.redT);
  int* redI = (int*)(smem + L.redI);
  SolveCol<T> P;
  P.n = n;
  P.Q = Q;
  P.q = q + c;
  P.qs = k;
  P.y0 = Y0 ? Y0 + c : nullptr;
  P.y = ws + c * 3 * n;
  P.g = P.y + n;
  P.w = P.g + n;
  P.x = X + c;
  P.s = s;
  P.trace = trace ? trace + c * 2 * trace_len : nullptr;
  P.trace_len = trace_len;
  solve_column<T, SW_NT>(P, tol, max_iter, iters + c, kkt + c, status + c,
                         rows_read ? rows_read + c : nullptr, lds_val, lds_idx, lds_val2,
                         lds_idx2, (T*)(smem + L.part), redT, redI);
}

size_t solve_wg_lds_bytes(int64_t n, int elem) { return sw_lds_layout(n, elem, SW_NT).total; }

template <typename T>
hipError_t launch_solve_wg(int64_t n, int64_t k, const T* Q, const T* q, const double* s,
                           double tol, int max_iter, const T* Y0, T* X, int32_t* iters,
                           double* kkt, int32_t* status, int64_t* rows_read, float* trace,
                           int trace_len, T* ws, hipStream_t st) {
  const size_t lds = solve_wg_lds_bytes(n, sizeof(T));
  hipError_t e = hipFuncSetAttribute((const void*)solve_wg_kernel<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(solve_wg_kernel<T>, dim3((unsigned)k), dim3(SW_NT), lds, st, n, k, Q, q, s,
                     tol, max_iter, Y0, X, iters, kkt, status, rows_read, trace, trace_len, ws);
  return hipGetLastError();
}
template hipError_t launch_solve_wg<float>(int64_t, int64_t, const float*, const float*,
                                          const double*, double, int, const float*, float*,
                                          int32_t*, double*, int32_t*, int64_t*, float*, int,
                                          float*, hipStream_t);
template hipError_t launch_solve_wg<double>(int64_t, int64_t, const double*, const double*,
                                           const double*, double, int, const double*, double*,
                                           int32_t*, double*, int32_t*, int64_t*, float*, int,
                                           double*, hipStream_t);

}  // namespace nnls
