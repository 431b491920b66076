// Uneven batch of independent problems (Algorithm 1 on each), run as one captured hipGraph:
//   queue reset -> batched Gram with fused rescale (gram.hip, one workgroup per problem) ->
//   batched solve: a grid of resident workgroups that take problems from an atomic queue in
//   longest-first order and run Algorithm 2 on each (solve_core.hpp), then x = y / s.
// The plan owns the graph; the caller owns every pool.  A launch of the plan is one graph
// launch on the caller's stream.
#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/nnls.h"
#include "solve_core.hpp"

namespace nnls {

struct BatchSolveArgs {
  const BatchDesc* desc;
  const int* order;  // problem indices, most expensive first
  int64_t count;
  int* counter;
  const float* Q_pool;
  const float* q_pool;
  const double* s_pool;
  float* X_pool;
  float* vec_pool;  // 3 floats per unknown: y, gradient, Q*gbar
  double tol;
  int max_iter;
  int32_t* iters;
  double* kkt;
  int32_t* status;
  int64_t* rows_read;
};

__global__ void batched_queue_reset(int* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

__global__ __launch_bounds__(SW_NT) void batched_solve_kernel(BatchSolveArgs B) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(B.counter, 1);
    __syncthreads();
    const int64_t idx = next;
    __syncthreads();
    if (idx >= B.count) break;  // uniform: every thread read the same value
    const int p = B.order[idx];
    const BatchDesc D = B.desc[p];
    const SwLdsLayout L = sw_lds_layout(D.n, sizeof(float));
    SolveCol<float> P;
    P.n = D.n;
    P.Q = B.Q_pool + D.offQ;
    P.q = B.q_pool + D.offq;
    P.qs = 1;
    P.y0 = nullptr;
    P.y = B.vec_pool + 3 * D.offq;
    P.g = P.y + D.n;
    P.w = P.g + D.n;
    P.x = B.X_pool + D.offX;
    P.s = B.s_pool + D.offq;
    P.trace = nullptr;
    P.trace_len = 0;
    const int mi = B.max_iter > 0 ? B.max_iter : (int)(5 * D.n);
    solve_column<float>(P, B.tol, mi, B.iters + p, B.kkt + p, B.status + p,
                        B.rows_read ? B.rows_read + p : nullptr, (float*)(smem + L.val),
                        (int*)(smem + L.idx), (float*)(smem + L.val2), (int*)(smem + L.idx2),
                        (float*)(smem + L.redT), (int*)(smem + L.redI));
    __syncthreads();
  }
}

}  // namespace nnls

// ---- host side: the plan ----------------------------------------------------------------------
struct nnls_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t count = 0;
};

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct PlanLayout {
  size_t desc, order, counter, vec, total;
};

PlanLayout plan_layout(int64_t count, int64_t sum_n) {
  PlanLayout L;
  L.desc = 0;
  L.order = align256(L.desc + sizeof(nnls::BatchDesc) * count);
  L.counter = align256(L.order + sizeof(int) * count);
  L.vec = align256(L.counter + 256);
  L.total = align256(L.vec + sizeof(float) * 3 * sum_n);
  return L;
}

void plan_fail(hipError_t e) { nnls::record_hip_error(e); }

}  // namespace

extern "C" {

size_t nnls_batched_workspace_bytes(const nnls_problem_desc* host_desc, int64_t count) {
  if (!host_desc || count < 1) return 0;
  int64_t sum_n = 0;
  for (int64_t i = 0; i < count; ++i) sum_n += host_desc[i].n > 0 ? host_desc[i].n : 0;
  return plan_layout(count, sum_n).total;
}

int nnls_batched_plan_create(const nnls_problem_desc* host_desc, int64_t count, double tol,
                             int32_t max_iter, const float* A_pool, const float* B_pool,
                             float* Q_pool, float* q_pool, double* s_pool, float* X_pool,
                             int32_t* iters, double* kkt, int32_t* status, int64_t* rows_read,
                             void* ws, size_t ws_bytes, void* capture_stream, nnls_plan** out) {
  if (!out) return NNLS_E_ARG;
  *out = nullptr;
  if (!capture_stream) return NNLS_E_ARG;  // the null stream cannot be captured
  if (!host_desc || count < 1 || count > (1 << 30)) return NNLS_E_ARG;
  if (!A_pool || !B_pool || !Q_pool || !q_pool || !s_pool || !X_pool || !iters || !kkt ||
      !status)
    return NNLS_E_ARG;
  if (!(tol >= 0.0) || max_iter < 0) return NNLS_E_ARG;
  int64_t sum_n = 0, max_n = 0;
  for (int64_t i = 0; i < count; ++i) {
    const nnls_problem_desc& p = host_desc[i];
    if (p.d < 1 || p.n < 1 || p.offA < 0 || p.offB < 0 || p.offQ < 0 || p.offq < 0 || p.offX < 0)
      return NNLS_E_ARG;
    if (p.n > nnls::BATCH_MAX_N) return NNLS_E_UNSUPPORTED;
    sum_n += p.n;
    max_n = std::max<int64_t>(max_n, p.n);
  }
  const PlanLayout L = plan_layout(count, sum_n);
  if (!ws || ws_bytes < L.total) return NNLS_E_WORKSPACE;

  // device descriptors and the longest-first order (estimated cost: Gram d n^2 plus
  // iterations growing with n, each costing n^2)
  std::vector<nnls::BatchDesc> dd(count);
  std::vector<double> cost(count);
  for (int64_t i = 0; i < count; ++i) {
    const nnls_problem_desc& p = host_desc[i];
    dd[i] = nnls::BatchDesc{p.d, p.n, p.offA, p.offB, p.offQ, p.offq, p.offX, 0};
    cost[i] = (double)p.d * p.n * p.n + 2.0 * (double)p.n * p.n * (double)p.n / 2.0;
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

  char* base = (char*)ws;
  hipStream_t st = (hipStream_t)capture_stream;
  // one-time setup copies (blocking: the host vectors are released on return)
  hipError_t e = hipMemcpy(base + L.desc, dd.data(), sizeof(nnls::BatchDesc) * count,
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + L.order, order.data(), sizeof(int) * count, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }

  nnls::BatchSolveArgs B;
  B.desc = (const nnls::BatchDesc*)(base + L.desc);
  B.order = (const int*)(base + L.order);
  B.count = count;
  B.counter = (int*)(base + L.counter);
  B.Q_pool = Q_pool;
  B.q_pool = q_pool;
  B.s_pool = s_pool;
  B.X_pool = X_pool;
  B.vec_pool = (float*)(base + L.vec);
  B.tol = tol;
  B.max_iter = max_iter;
  B.iters = iters;
  B.kkt = kkt;
  B.status = status;
  B.rows_read = rows_read;

  const size_t solve_lds = nnls::sw_lds_layout(max_n, sizeof(float)).total;
  int dev = 0, cus = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  e = hipFuncSetAttribute((const void*)nnls::batched_solve_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)solve_lds);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, (const void*)nnls::batched_solve_kernel, nnls::SW_NT, solve_lds);
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }
  const int64_t grid = std::min<int64_t>(count, (int64_t)cus * std::max(per_cu, 1));

  e = nnls::prepare_batched_gram();  // kernel attributes are set outside the capture
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }
  nnls_plan* plan = new (std::nothrow) nnls_plan();
  if (!plan) return NNLS_E_HIP;
  plan->count = count;
  e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(nnls::batched_queue_reset, dim3(1), dim3(64), 0, st, B.counter);
    hipError_t e1 = nnls::launch_batched_gram(B.desc, count, A_pool, B_pool, Q_pool, q_pool,
                                              s_pool, st);
    hipLaunchKernelGGL(nnls::batched_solve_kernel, dim3((unsigned)grid), dim3(nnls::SW_NT),
                       solve_lds, st, B);
    hipError_t e2 = hipGetLastError();
    e = hipStreamEndCapture(st, &plan->graph);
    if (e == hipSuccess && e1 != hipSuccess) e = e1;
    if (e == hipSuccess && e2 != hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_fail(e);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return NNLS_E_HIP;
  }
  *out = plan;
  return NNLS_OK;
}

int nnls_batched_plan_launch(nnls_plan* plan, void* stream) {
  if (!plan || !plan->exec) return NNLS_E_ARG;
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

void nnls_batched_plan_destroy(nnls_plan* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

}  // extern "C"
