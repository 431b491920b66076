// C ABI of libnnls: argument validation, workspace sizing and dispatch to the HIP kernels.
// Every check runs on the host before the first HIP call, so argument errors never touch the
// device.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/nnls.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_last_hip_error;

int hip_fail(hipError_t e) {
  g_last_hip_error = hipGetErrorString(e);
  return NNLS_E_HIP;
}

}  // namespace

void nnls::record_hip_error(hipError_t e) { g_last_hip_error = hipGetErrorString(e); }

int nnls::spin_limit_setting() {
  const char* v = getenv("NNLS_SPIN_LIMIT");
  if (v != nullptr && *v != '\0') {
    char* end = nullptr;
    const long x = strtol(v, &end, 10);
    if (end != v && *end == '\0' && x >= 0 && x <= (1L << 24)) return (int)x;
  }
  return 1 << 24;
}

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Largest LDS the one-workgroup-per-column solver may request on gfx950 (160 KiB per CU).
constexpr size_t kMaxLds = 160 * 1024;

bool valid_dtype(int dt) { return dt == NNLS_F32 || dt == NNLS_F64; }
size_t elem_size(int dt) { return dt == NNLS_F64 ? 8 : 4; }

size_t gram_ws(int64_t d, int64_t n, int64_t k, int mode) {
  return align_up(mode == NNLS_GRAM_BF16X3 ? nnls::gram_bf16x3_ws_bytes(d, n, k) : 0);
}

// The scale pass and the Gram run one after the other on the stream, so they share the buffer.
size_t prepare_ws(int64_t d, int64_t n, int64_t k, int mode) {
  if (mode == NNLS_GRAM_BF16X3) return align_up(nnls::prepare_bf16x3_ws_bytes(d, n, k));
  size_t a = align_up(nnls::colnorm_ws_bytes(d, n));
  size_t b = gram_ws(d, n, k, mode);
  return a > b ? a : b;
}

// Solver choice (FP32):
//   one right-hand side with n >= kPersistentMinN  -> whole-GPU kernel, Q held in registers
//                                                     (n <= 5120) or streamed (larger n)
//   several right-hand sides, n small enough for LDS -> matrix-core many-RHS kernel
//   otherwise (and FP64)                             -> one workgroup per column
// NNLS_SOLVER=wg|persistent|regq|mrhs in the environment forces a choice where it is valid.
constexpr int64_t kPersistentMinN = 1536;

enum SolverKind { SOLVER_WG = 0, SOLVER_PERSISTENT = 1, SOLVER_MRHS = 2, SOLVER_REGQ = 3 };

int solver_override() {
  const char* v = getenv("NNLS_SOLVER");
  if (!v) return -1;
  if (strcmp(v, "wg") == 0) return SOLVER_WG;
  if (strcmp(v, "persistent") == 0) return SOLVER_PERSISTENT;
  if (strcmp(v, "mrhs") == 0) return SOLVER_MRHS;
  if (strcmp(v, "regq") == 0) return SOLVER_REGQ;
  return -1;
}

SolverKind pick_solver(int64_t n, int64_t k, int dt) {
  const bool can_p = dt == NNLS_F32 && nnls::solve_persistent_supported(n, k);
  const bool can_r = dt == NNLS_F32 && nnls::solve_regq_supported(n, k);
  const bool can_m = dt == NNLS_F32 && nnls::solve_mrhs_supported(n, k);
  const bool can_w = nnls::solve_wg_lds_bytes(n, (int)elem_size(dt)) <= kMaxLds;
  const int o = solver_override();
  if (o == SOLVER_PERSISTENT && can_p) return SOLVER_PERSISTENT;
  if (o == SOLVER_REGQ && can_r) return SOLVER_REGQ;
  if (o == SOLVER_MRHS && can_m) return SOLVER_MRHS;
  if (o == SOLVER_WG && can_w) return SOLVER_WG;
  if (can_r && (n >= kPersistentMinN || !can_w)) return SOLVER_REGQ;
  if (can_p && (n >= kPersistentMinN || !can_w)) return SOLVER_PERSISTENT;
  if (can_m) return SOLVER_MRHS;
  return SOLVER_WG;
}

bool solver_supported(int64_t n, int64_t k, int dt) {
  return (dt == NNLS_F32 && nnls::solve_persistent_supported(n, k)) ||
         (dt == NNLS_F32 && nnls::solve_regq_supported(n, k)) ||
         (dt == NNLS_F32 && nnls::solve_mrhs_supported(n, k)) ||
         nnls::solve_wg_lds_bytes(n, (int)elem_size(dt)) <= kMaxLds;
}

size_t solve_ws(int64_t n, int64_t k, int dt) {
  switch (pick_solver(n, k, dt)) {
    case SOLVER_PERSISTENT:
      return align_up(nnls::solve_persistent_ws_bytes(n));
    case SOLVER_REGQ:
      return align_up(nnls::solve_regq_ws_bytes(n));
    case SOLVER_MRHS:
      return align_up(nnls::solve_mrhs_ws_bytes());
    default:
      return align_up(elem_size(dt) * 3 * n * k);
  }
}

// ---- scratch of the solve that allocates nothing ------------------------------------------
// One copy per GPU the library runs on, held until the process ends.  In host code `scratch` is
// a host-side stand-in, not a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[NNLS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

hipError_t scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* nnls_last_hip_error(void) { return g_last_hip_error.c_str(); }

const char* nnls_solver_name(int64_t n, int64_t k, int dtype) {
  if (n < 1 || k < 1 || !valid_dtype(dtype) || !solver_supported(n, k, dtype)) return "";
  switch (pick_solver(n, k, dtype)) {
    case SOLVER_REGQ: return "regq";
    case SOLVER_PERSISTENT: return "persistent";
    case SOLVER_MRHS: return "mrhs";
    default: return "wg";
  }
}

const char* nnls_version(void) { return "nnls-mi355x 0.1 (gfx950)"; }

size_t nnls_workspace_bytes(int op, int64_t d, int64_t n, int64_t k, int mode, int dtype) {
  if (n < 1 || k < 0 || !valid_dtype(dtype)) return 0;
  switch (op) {
    case NNLS_OP_PREPARE:
      if (d < 1) return 0;
      return prepare_ws(d, n, k, mode);
    case NNLS_OP_SOLVE:
      return k < 1 ? 0 : solve_ws(n, k, dtype);
    case NNLS_OP_REFINE:
      return (d < 1 || k < 1) ? 0 : align_up(nnls::refine_ws_bytes(d, n, k));
    case NNLS_OP_SCALES:
      return d < 1 ? 0 : align_up(nnls::colnorm_ws_bytes(d, n));
    case NNLS_OP_GRAM:
      return d < 1 ? 0 : gram_ws(d, n, k, mode);
    default:
      return 0;
  }
}

static int validate_scales(int64_t d, int64_t n, const void* A, int64_t lda, int dtype,
                           const double* s) {
  if (d < 1 || n < 1 || !valid_dtype(dtype)) return NNLS_E_ARG;
  if (!A || !s || lda < n) return NNLS_E_ARG;
  if (n > (int64_t)1 << 30 || d > ((int64_t)1 << 40) / n) return NNLS_E_UNSUPPORTED;
  return NNLS_OK;
}

static int validate_gram(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda,
                         const void* B, int64_t ldb, int mode, int dtype, const void* Q,
                         const void* q) {
  if (d < 1 || n < 1 || k < 0) return NNLS_E_ARG;
  if (!valid_dtype(dtype)) return NNLS_E_ARG;
  if (dtype == NNLS_F64 && mode != NNLS_GRAM_FP64) return NNLS_E_ARG;
  if (dtype == NNLS_F32 && mode != NNLS_GRAM_FP32 && mode != NNLS_GRAM_BF16X3) return NNLS_E_ARG;
  if (!A || !Q || lda < n) return NNLS_E_ARG;
  if (k > 0 && (!B || !q || ldb < k)) return NNLS_E_ARG;
  if (n > (int64_t)1 << 30 || d > ((int64_t)1 << 40) / n) return NNLS_E_UNSUPPORTED;
  return NNLS_OK;
}

static hipError_t run_scales(int64_t d, int64_t n, const void* A, int64_t lda, int dtype,
                             double* s, void* ws, hipStream_t st) {
  if (dtype == NNLS_F64)
    return nnls::launch_colnorm<double>(d, n, (const double*)A, lda, s, (double*)ws, st);
  return nnls::launch_colnorm<float>(d, n, (const float*)A, lda, s, (double*)ws, st);
}

static hipError_t run_gram(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda,
                           const void* B, int64_t ldb, int mode, int dtype, const double* s,
                           void* Q, void* q, void* ws, hipStream_t st) {
  if (dtype == NNLS_F64)
    return nnls::launch_gram_fma<double>(d, n, k, (const double*)A, lda, (const double*)B, ldb,
                                         s, (double*)Q, (double*)q, st);
  if (mode == NNLS_GRAM_BF16X3)
    return nnls::launch_gram_bf16x3(d, n, k, (const float*)A, lda, (const float*)B, ldb, s,
                                    (float*)Q, (float*)q, (float*)ws, st);
  return nnls::launch_gram_fma<float>(d, n, k, (const float*)A, lda, (const float*)B, ldb, s,
                                      (float*)Q, (float*)q, st);
}

int nnls_column_scales(int64_t d, int64_t n, const void* A, int64_t lda, int dtype, double* s,
                       void* ws, size_t ws_bytes, void* stream) {
  int rc = validate_scales(d, n, A, lda, dtype, s);
  if (rc != NNLS_OK) return rc;
  const size_t need = align_up(nnls::colnorm_ws_bytes(d, n));
  if (ws_bytes < need || !ws) return NNLS_E_WORKSPACE;
  hipError_t e = run_scales(d, n, A, lda, dtype, s, ws, (hipStream_t)stream);
  return e == hipSuccess ? NNLS_OK : hip_fail(e);
}

int nnls_gram_rescaled(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda,
                       const void* B, int64_t ldb, int mode, int dtype, const double* s, void* Q,
                       void* q, void* ws, size_t ws_bytes, void* stream) {
  int rc = validate_gram(d, n, k, A, lda, B, ldb, mode, dtype, Q, q);
  if (rc != NNLS_OK) return rc;
  if (!s) return NNLS_E_ARG;
  const size_t need = gram_ws(d, n, k, mode);
  if (ws_bytes < need || (need > 0 && !ws)) return NNLS_E_WORKSPACE;
  hipError_t e = run_gram(d, n, k, A, lda, B, ldb, mode, dtype, s, Q, q, ws, (hipStream_t)stream);
  return e == hipSuccess ? NNLS_OK : hip_fail(e);
}

int nnls_gram(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
              int64_t ldb, int mode, int dtype, void* H, void* h, void* ws, size_t ws_bytes,
              void* stream) {
  int rc = validate_gram(d, n, k, A, lda, B, ldb, mode, dtype, H, h);
  if (rc != NNLS_OK) return rc;
  const size_t need = gram_ws(d, n, k, mode);
  if (ws_bytes < need || (need > 0 && !ws)) return NNLS_E_WORKSPACE;
  hipError_t e = run_gram(d, n, k, A, lda, B, ldb, mode, dtype, nullptr, H, h, ws,
                          (hipStream_t)stream);
  return e == hipSuccess ? NNLS_OK : hip_fail(e);
}

int nnls_prepare(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                 int64_t ldb, int mode, int dtype, void* Q, void* q, double* s, void* ws,
                 size_t ws_bytes, void* stream) {
  int rc = validate_gram(d, n, k, A, lda, B, ldb, mode, dtype, Q, q);
  if (rc != NNLS_OK) return rc;
  if (!s) return NNLS_E_ARG;
  const size_t need = prepare_ws(d, n, k, mode);
  if (ws_bytes < need || (need > 0 && !ws)) return NNLS_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (dtype == NNLS_F32 && mode == NNLS_GRAM_BF16X3) {
    e = nnls::launch_prepare_bf16x3(d, n, k, (const float*)A, lda, (const float*)B, ldb, s,
                                    (float*)Q, (float*)q, ws, st);
    return e == hipSuccess ? NNLS_OK : hip_fail(e);
  }
  e = run_scales(d, n, A, lda, dtype, s, ws, st);
  if (e != hipSuccess) return hip_fail(e);
  e = run_gram(d, n, k, A, lda, B, ldb, mode, dtype, s, Q, q, ws, st);
  return e == hipSuccess ? NNLS_OK : hip_fail(e);
}

// Host checks of a solve (every argument but the workspace).
static int validate_solve(int64_t n, int64_t k, int dtype, const void* Q, const void* q,
                          double tol, int32_t max_iter, const void* X, const int32_t* iters,
                          const double* kkt, const int32_t* status, const float* trace,
                          int32_t trace_len) {
  if (n < 1 || k < 1 || !valid_dtype(dtype)) return NNLS_E_ARG;
  if (!Q || !q || !X || !iters || !kkt || !status) return NNLS_E_ARG;
  if (trace_len < 0 || (trace != nullptr && trace_len == 0)) return NNLS_E_ARG;
  if (trace != nullptr && k * (int64_t)trace_len > ((int64_t)1 << 40)) return NNLS_E_UNSUPPORTED;
  if (!(tol >= 0.0) || !isfinite(tol) || max_iter < 0) return NNLS_E_ARG;
  if (n > (int64_t)1 << 30 || k > (int64_t)1 << 31) return NNLS_E_UNSUPPORTED;
  if (!solver_supported(n, k, dtype)) return NNLS_E_UNSUPPORTED;
  return NNLS_OK;
}

// The solver launch of a validated solve, with its scratch state in ws.
static int run_solve(int64_t n, int64_t k, int dtype, const void* Q, const void* q,
                     const double* s, double tol, int32_t max_iter, const void* Y0, void* X,
                     int32_t* iters, double* kkt, int32_t* status, int64_t* rows_read,
                     float* trace, int32_t trace_len, void* ws, hipStream_t st) {
  const int tl = trace != nullptr ? trace_len : 0;
  const int mi = max_iter == 0 ? (int)(5 * n < (1 << 30) ? 5 * n : (1 << 30)) : max_iter;
  hipError_t e;
  const SolverKind kind = pick_solver(n, k, dtype);
  if (kind == SOLVER_MRHS) {
    if (((uintptr_t)Q & 15) != 0) return NNLS_E_ARG;  // rows are read as 16-byte vectors
    e = nnls::launch_solve_mrhs(n, k, (const float*)Q, (const float*)q, s, tol, mi,
                                (const float*)Y0, (float*)X, iters, kkt, status, rows_read, trace,
                                tl, ws, st);
  } else if (kind == SOLVER_REGQ) {
    e = nnls::launch_solve_regq(n, (const float*)Q, (const float*)q, s, tol, mi,
                                (const float*)Y0, (float*)X, iters, kkt, status, rows_read, trace,
                                tl, ws, st);
  } else if (kind == SOLVER_PERSISTENT) {
    if (((uintptr_t)Q & 15) != 0) return NNLS_E_ARG;  // rows are read as 16-byte vectors
    e = nnls::launch_solve_persistent(n, (const float*)Q, (const float*)q, s, tol, mi,
                                      (const float*)Y0, (float*)X, iters, kkt, status,
                                      rows_read, trace, tl, ws, st);
  } else if (dtype == NNLS_F64)
    e = nnls::launch_solve_wg<double>(n, k, (const double*)Q, (const double*)q, s, tol, mi,
                                      (const double*)Y0, (double*)X, iters, kkt, status,
                                      rows_read, trace, tl, (double*)ws, st);
  else
    e = nnls::launch_solve_wg<float>(n, k, (const float*)Q, (const float*)q, s, tol, mi,
                                     (const float*)Y0, (float*)X, iters, kkt, status, rows_read,
                                     trace, tl, (float*)ws, st);
  if (e != hipSuccess) return hip_fail(e);
  return NNLS_OK;
}

int nnls_prepare_split(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                       const float* B, int64_t ldb, double* s, void* ws, size_t ws_bytes,
                       void* stream) {
  const float* fake_q = k > 0 ? (const float*)B : nullptr;  // Q, q are not written here
  int rc = validate_gram(d, n, k, A, lda, B, ldb, NNLS_GRAM_BF16X3, NNLS_F32, A, fake_q);
  if (rc != NNLS_OK) return rc;
  if (!s) return NNLS_E_ARG;
  const size_t need = prepare_ws(d, n, k, NNLS_GRAM_BF16X3);
  if (ws_bytes < need || !ws) return NNLS_E_WORKSPACE;
  hipError_t e = nnls::launch_prepare_split_bf16x3(d, n, k, A, lda, B, ldb, s, ws,
                                                   (hipStream_t)stream);
  return e == hipSuccess ? NNLS_OK : hip_fail(e);
}

int nnls_prepare_product(int64_t d, int64_t n, int64_t k, const double* s, float* Q, float* q,
                         void* ws, size_t ws_bytes, void* stream) {
  if (d < 1 || n < 1 || k < 0 || !s || !Q || (k > 0 && !q)) return NNLS_E_ARG;
  if (n > (int64_t)1 << 30 || d > ((int64_t)1 << 40) / n) return NNLS_E_UNSUPPORTED;
  const size_t need = prepare_ws(d, n, k, NNLS_GRAM_BF16X3);
  if (ws_bytes < need || !ws) return NNLS_E_WORKSPACE;
  hipError_t e = nnls::launch_prepare_product_bf16x3(d, n, k, s, Q, q, ws, (hipStream_t)stream);
  return e == hipSuccess ? NNLS_OK : hip_fail(e);
}

int nnls_solve(int64_t n, int64_t k, int dtype, const void* Q, const void* q, const double* s,
               double tol, int32_t max_iter, const void* Y0, void* X, int32_t* iters,
               double* kkt, int32_t* status, int64_t* rows_read, float* trace,
               int32_t trace_len, void* ws, size_t ws_bytes, void* stream) {
  const int rc = validate_solve(n, k, dtype, Q, q, tol, max_iter, X, iters, kkt, status, trace,
                                trace_len);
  if (rc != NNLS_OK) return rc;
  const size_t need = solve_ws(n, k, dtype);
  if (ws_bytes < need || !ws) return NNLS_E_WORKSPACE;
  return run_solve(n, k, dtype, Q, q, s, tol, max_iter, Y0, X, iters, kkt, status, rows_read,
                   trace, trace_len, ws, (hipStream_t)stream);
}

int nnls_solve_noalloc(int64_t n, int64_t k, int dtype, const void* Q, const void* q,
                       const double* s, double tol, int32_t max_iter, const void* Y0, void* X,
                       int32_t* iters, double* kkt, int32_t* status, int64_t* rows_read,
                       float* trace, int32_t trace_len, void* stream) {
  const int rc = validate_solve(n, k, dtype, Q, q, tol, max_iter, X, iters, kkt, status, trace,
                                trace_len);
  if (rc != NNLS_OK) return rc;
  if (solve_ws(n, k, dtype) > (size_t)NNLS_NOALLOC_SCRATCH_BYTES) return NNLS_E_WORKSPACE;
  void* ws = nullptr;
  const hipError_t e = scratch_of_current_device(&ws);
  if (e != hipSuccess) return hip_fail(e);
  return run_solve(n, k, dtype, Q, q, s, tol, max_iter, Y0, X, iters, kkt, status, rows_read,
                   trace, trace_len, ws, (hipStream_t)stream);
}

int nnls_refine(int64_t d, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                int64_t ldb, int dtype, void* X, double* kkt64, double* obj64, void* ws,
                size_t ws_bytes, void* stream) {
  if (d < 1 || n < 1 || k < 1 || !valid_dtype(dtype)) return NNLS_E_ARG;
  if (!A || !B || !X || !kkt64 || lda < n || ldb < k) return NNLS_E_ARG;
  if (n > (int64_t)1 << 30 || k > (int64_t)1 << 31) return NNLS_E_UNSUPPORTED;
  const size_t need = align_up(nnls::refine_ws_bytes(d, n, k));
  if (ws_bytes < need || !ws) return NNLS_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (dtype == NNLS_F64)
    e = nnls::launch_refine<double>(d, n, k, (const double*)A, lda, (const double*)B, ldb,
                                    (double*)X, kkt64, obj64, ws, st);
  else
    e = nnls::launch_refine<float>(d, n, k, (const float*)A, lda, (const float*)B, ldb,
                                   (float*)X, kkt64, obj64, ws, st);
  if (e != hipSuccess) return hip_fail(e);
  return NNLS_OK;
}

}  // extern "C"
