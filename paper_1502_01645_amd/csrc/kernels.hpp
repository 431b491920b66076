// Internal launchers of the NNLS kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nnls {

constexpr int NNLS_CONVERGED_DEV = 0;
constexpr int NNLS_MAXITER_DEV = 1;
constexpr int NNLS_BREAKDOWN_DEV = 2;
constexpr int NNLS_NONFINITE_DEV = 3;
constexpr int NNLS_FELL_BACK_DEV = 4;

// Remembers the text of a failed HIP call for nnls_last_hip_error (capi.hip).
void record_hip_error(hipError_t e);

// Poll limit of every wait of the whole-GPU solvers (capi.hip): 1 << 24, a bound no normal
// launch reaches, or NNLS_SPIN_LIMIT from the environment, a test hook that forces the give-up
// path (every wait still ends, the solve reports BREAKDOWN with iters = -1).
int spin_limit_setting();

// One problem of an uneven batch (device copy of the caller's descriptor): A is [d, n] at
// A_pool + offA, b is [d] at B_pool + offB, Q is [n, n] at Q_pool + offQ, q, s and x are [n] at
// offset offq of their pools (s in the FP64 pool), x at X_pool + offX.
struct BatchDesc {
  int64_t d, n, offA, offB, offQ, offq, offX, pad;
};

// gram.hip
size_t colnorm_ws_bytes(int64_t d, int64_t n);
template <typename T>
hipError_t launch_colnorm(int64_t d, int64_t n, const T* A, int64_t lda, double* s, double* ws,
                          hipStream_t st);
size_t gram_bf16x3_ws_bytes(int64_t d, int64_t n, int64_t k);
// Column norms and the BF16x3 Gram in one pass over A (the norms come from the operand split).
size_t prepare_bf16x3_ws_bytes(int64_t d, int64_t n, int64_t k);
hipError_t launch_prepare_bf16x3(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                                 const float* B, int64_t ldb, double* s, float* Q, float* q,
                                 void* ws, hipStream_t st);
// launch_prepare_bf16x3 in its two steps: the operand split with the column norms, then the
// product from the split planes left in ws.
hipError_t launch_prepare_split_bf16x3(int64_t d, int64_t n, int64_t k, const float* A,
                                       int64_t lda, const float* B, int64_t ldb, double* s,
                                       void* ws, hipStream_t st);
hipError_t launch_prepare_product_bf16x3(int64_t d, int64_t n, int64_t k, const double* s,
                                         float* Q, float* q, void* ws, hipStream_t st);
hipError_t launch_gram_bf16x3(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                              const float* B, int64_t ldb, const double* s, float* Q, float* q,
                              float* ws, hipStream_t st);
template <typename T>
hipError_t launch_gram_fma(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
                           int64_t ldb, const double* s, T* Q, T* q, hipStream_t st);

constexpr int64_t BATCH_MAX_N = 1024;
// One tile (ti, tj), ti <= tj, of problem p's [A | b]^T [A | b] in the batched Gram.
struct BatchGramItem {
  int32_t p;
  int16_t ti, tj;
};
size_t batched_gram_lds_bytes(int bm);
hipError_t prepare_batched_gram();
// The tiles of `items` (diagonal tiles when diag, else tiles above the diagonal, which need the
// scales the diagonal launch wrote), at tile size bm = 64 or 128.
hipError_t launch_batched_gram(int bm, bool diag, const BatchGramItem* items, int64_t count,
                               const BatchDesc* desc, const float* A_pool, const float* B_pool,
                               float* Q_pool, float* q_pool, double* s_pool, hipStream_t st);

// solve_wg.hip
size_t solve_wg_lds_bytes(int64_t n, int elem);
// Every solver launcher takes the per-update trace: trace [k][trace_len][2] FP32 (r of the
// iterate after t updates, ||gbar||^2 of it) for t < trace_len, or nullptr.
template <typename T>
hipError_t launch_solve_wg(int64_t n, int64_t k, const T* Q, const T* q, const double* s,
                           double tol, int max_iter, const T* Y0, T* X, int32_t* iters,
                           double* kkt, int32_t* status, int64_t* rows_read, float* trace,
                           int trace_len, T* ws, hipStream_t st);

// solve_regq.hip (one right-hand side, Q held in the register file of the whole GPU)
bool solve_regq_supported(int64_t n, int64_t k);
size_t solve_regq_ws_bytes(int64_t n);
hipError_t launch_solve_regq(int64_t n, const float* Q, const float* q, const double* s,
                             double tol, int max_iter, const float* Y0, float* X, int32_t* iters,
                             double* kkt, int32_t* status, int64_t* rows_read, float* trace,
                             int trace_len, void* ws, hipStream_t st);

// solve_persistent.hip
bool solve_persistent_supported(int64_t n, int64_t k);
size_t solve_persistent_ws_bytes(int64_t n);
hipError_t launch_solve_persistent(int64_t n, const float* Q, const float* q, const double* s,
                                   double tol, int max_iter, const float* Y0, float* X,
                                   int32_t* iters, double* kkt, int32_t* status,
                                   int64_t* rows_read, float* trace, int trace_len, void* ws,
                                   hipStream_t st);

// solve_mrhs.hip
bool solve_mrhs_supported(int64_t n, int64_t k);
size_t solve_mrhs_ws_bytes();
hipError_t launch_solve_mrhs(int64_t n, int64_t k, const float* Q, const float* q,
                             const double* s, double tol, int max_iter, const float* Y0,
                             float* X, int32_t* iters, double* kkt, int32_t* status,
                             int64_t* rows_read, float* trace, int trace_len, void* ws,
                             hipStream_t st);

// refine.hip
size_t refine_ws_bytes(int64_t d, int64_t n, int64_t k);
template <typename T>
hipError_t launch_refine(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
                         int64_t ldb, T* X, double* kkt64, double* obj64, void* ws,
                         hipStream_t st);

}  // namespace nnls
