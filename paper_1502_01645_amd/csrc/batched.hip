// Uneven batch of independent problems (Algorithm 1 on each), run as one captured hipGraph:
//   queue reset -> batched Gram with fused rescale (gram.hip: the diagonal tiles of every
//   problem, then the tiles above the diagonal) -> batched solve: per thread-count class a grid
//   of resident workgroups that take the class's problems from an atomic queue in longest-first
//   order and run Algorithm 2 on each (solve_core.hpp), then x = y / s; the classes are parallel
//   branches of the graph.
// Problems fall in size classes by n; each class has a Gram tile size (64 or 128) and a solver
// workgroup size (256, 512 or 1024 threads).  nnls_autotune measures both per class on
// synthetic problems of the caller's shapes and records the fastest in a JSON cache that
// nnls_batched_plan_create reads.  The plan owns the graph; the caller owns every pool.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/nnls.h"
#include "solve_core.hpp"

namespace nnls {

struct BatchSolveArgs {
  const BatchDesc* desc;
  const int* order;  // problem indices of this class, most expensive first
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

constexpr int kSolveClasses = 3;
constexpr int kSolveThreads[kSolveClasses] = {256, 512, 1024};
// A solve group is a (workgroup size, resident-per-CU cap) pair: one persistent launch each.
constexpr int kCaps = 2;  // cap index 0: as many as fit; 1: one per compute unit
constexpr int kSolveGroups = kSolveClasses * kCaps;

__global__ void batched_queue_reset(int* counters, int count) {
  if ((int)threadIdx.x < count) counters[threadIdx.x * 64] = 0;
}

template <int NT>
__global__ __launch_bounds__(NT) void batched_solve_kernel(BatchSolveArgs B) {
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
    const SwLdsLayout L = sw_lds_layout(D.n, sizeof(float), NT);
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
    solve_column<float, NT>(P, B.tol, mi, B.iters + p, B.kkt + p, B.status + p,
                            B.rows_read ? B.rows_read + p : nullptr, (float*)(smem + L.val),
                            (int*)(smem + L.idx), (float*)(smem + L.val2), (int*)(smem + L.idx2),
                            (float*)(smem + L.part), (float*)(smem + L.redT),
                            (int*)(smem + L.redI));
    __syncthreads();
  }
}

// ---- synthetic problems for the autotuner ----------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", 2014):
// the output of the generator seeded with `key`, as a uniform double in [0, 1).
__device__ __forceinline__ double tune_u01(uint64_t key) {
  uint64_t z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ uint64_t tune_key(int64_t p, int64_t i, int stream) {
  return ((uint64_t)p << 40) ^ ((uint64_t)i << 2) ^ (uint64_t)stream;
}

// Problem p (one workgroup): A U[0, 1], x 60 % zeros else U[0, 1], b = A x + 1 % noise.
__global__ __launch_bounds__(256) void tune_problem_kernel(const BatchDesc* __restrict__ desc,
                                                           float* __restrict__ A_pool,
                                                           float* __restrict__ B_pool) {
  const int64_t p = blockIdx.x;
  const BatchDesc D = desc[p];
  float* A = A_pool + D.offA;
  for (int64_t e = threadIdx.x; e < D.d * D.n; e += 256) A[e] = (float)tune_u01(tune_key(p, e, 0));
  __syncthreads();
  for (int64_t r = threadIdx.x; r < D.d; r += 256) {
    double acc = 0.0;
    for (int64_t j = 0; j < D.n; ++j) {
      const double xj = tune_u01(tune_key(p, j, 1)) < 0.6 ? 0.0 : tune_u01(tune_key(p, j, 2));
      acc += (double)A[r * D.n + j] * xj;
    }
    B_pool[D.offB + r] = (float)(acc * (1.0 + 0.02 * (tune_u01(tune_key(p, r, 3)) - 0.5)));
  }
}

}  // namespace nnls

// ---- host side -------------------------------------------------------------------------------
struct nnls_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t count = 0;
};

namespace {

using nnls::BatchDesc;
using nnls::BatchGramItem;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Size classes by n: class c holds kClassHi[c - 1] < n <= kClassHi[c].
constexpr int kClasses = 5;
constexpr int64_t kClassHi[kClasses] = {64, 128, 256, 512, 1024};
int size_class(int64_t n) {
  for (int c = 0; c < kClasses; ++c)
    if (n <= kClassHi[c]) return c;
  return kClasses - 1;
}

struct ClassParams {
  int gram_tile;      // 64 or 128
  int solve_threads;  // 256, 512 or 1024
  int solve_per_cu;   // resident solver workgroups per compute unit: 0 = as many as fit, else
                      // this cap (fewer problems in flight keep their Q in the caches)
};
// Without a tuning record: 128-wide Gram tiles and 256-thread solver workgroups everywhere,
// as many resident as fit.
constexpr ClassParams kDefault = {128, 256, 0};
constexpr int kPerCuCaps[nnls::kCaps] = {0, 1};
int cap_index(int cap) { return cap == 1 ? 1 : 0; }

int solve_slot(int nt) {
  for (int i = 0; i < nnls::kSolveClasses; ++i)
    if (nnls::kSolveThreads[i] == nt) return i;
  return -1;
}

// Gram tiles (ti, tj), ti <= tj, of one problem at tile size bm: ti < ceil(n / bm) (rows of A),
// tj < ceil((n + 1) / bm) (columns of [A | b]).
void problem_items(int32_t p, int64_t n, int bm, std::vector<BatchGramItem>& diag,
                   std::vector<BatchGramItem>& off) {
  const int T = (int)((n + bm - 1) / bm), Ta = (int)((n + 1 + bm - 1) / bm);
  for (int ti = 0; ti < T; ++ti) {
    diag.push_back(BatchGramItem{p, (int16_t)ti, (int16_t)ti});
    for (int tj = ti + 1; tj < Ta; ++tj) off.push_back(BatchGramItem{p, (int16_t)ti, (int16_t)tj});
  }
}

int64_t item_bound(int64_t n) {  // tiles at the smaller tile size, an upper bound for both
  const int64_t T = (n + 63) / 64, Ta = (n + 64) / 64;
  return T * Ta - T * (T - 1) / 2;
}

// Estimated cost of a problem for the longest-first order: Gram d n^2 plus iterations growing
// with n, each costing n^2.
double problem_cost(int64_t d, int64_t n) {
  return (double)d * n * n + (double)n * n * (double)n;
}

struct PlanLayout {
  size_t desc, items, order, counter, vec, total;
};

PlanLayout plan_layout(int64_t count, int64_t sum_n, int64_t max_items) {
  PlanLayout L;
  L.desc = 0;
  L.items = align256(L.desc + sizeof(BatchDesc) * count);
  L.order = align256(L.items + sizeof(BatchGramItem) * max_items);
  L.counter = align256(L.order + sizeof(int) * count);
  L.vec = align256(L.counter + sizeof(int) * 64 * nnls::kSolveGroups);
  L.total = align256(L.vec + sizeof(float) * 3 * sum_n);
  return L;
}

void plan_fail(hipError_t e) { nnls::record_hip_error(e); }

// ---- the tuning cache (JSON, one entry per line) ----------------------------------------------
std::mutex g_tune_mu;  // guards reads and writes of cache files in this process

struct TuneEntry {
  std::string arch, op, dtype;
  int64_t lo = 0, hi = 0;
  int gram_tile = 0, solve_threads = 0, solve_per_cu = 0;
  std::string line;  // the entry as written
};

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "";
  return std::string(prop.gcnArchName);
}

bool json_str(const std::string& s, const char* key, std::string& out) {
  const std::string k = std::string("\"") + key + "\": \"";
  const size_t a = s.find(k);
  if (a == std::string::npos) return false;
  const size_t b = s.find('"', a + k.size());
  if (b == std::string::npos) return false;
  out = s.substr(a + k.size(), b - a - k.size());
  return true;
}

bool json_int(const std::string& s, const char* key, int64_t& out) {
  const std::string k = std::string("\"") + key + "\": ";
  const size_t a = s.find(k);
  if (a == std::string::npos) return false;
  char* end = nullptr;
  const long long v = strtoll(s.c_str() + a + k.size(), &end, 10);
  if (end == s.c_str() + a + k.size()) return false;
  out = (int64_t)v;
  return true;
}

// Entries of a cache file (unreadable lines are skipped; a missing file has none).
std::vector<TuneEntry> read_cache(const char* path) {
  std::vector<TuneEntry> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  std::string line;
  int c;
  while (true) {
    line.clear();
    while ((c = fgetc(f)) != EOF && c != '\n') line.push_back((char)c);
    if (line.find("\"op\": ") != std::string::npos) {
      TuneEntry e;
      int64_t gt = 0, st = 0, pc = 0;
      if (json_str(line, "arch", e.arch) && json_str(line, "op", e.op) &&
          json_str(line, "dtype", e.dtype) && json_int(line, "n_lo", e.lo) &&
          json_int(line, "n_hi", e.hi) && json_int(line, "gram_tile", gt) &&
          json_int(line, "solve_threads", st)) {
        if (!json_int(line, "solve_wgs_per_cu", pc)) pc = 0;
        e.gram_tile = (int)gt;
        e.solve_threads = (int)st;
        e.solve_per_cu = (int)pc;
        e.line = line;
        while (!e.line.empty() && (e.line.back() == ',' || e.line.back() == ' '))
          e.line.pop_back();
        out.push_back(e);
      }
    }
    if (c == EOF) break;
  }
  fclose(f);
  return out;
}

bool write_cache(const char* path, const std::vector<TuneEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\"format\": \"nnls-autotune-1\", \"entries\": [\n");
  for (size_t i = 0; i < entries.size(); ++i)
    fprintf(f, "%s%s\n", entries[i].line.c_str(), i + 1 < entries.size() ? "," : "");
  fprintf(f, "]}\n");
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return false;
  }
  return true;
}

// Per-class parameters for this device: the cache's entries for (arch, "batched", "f32", class
// bounds), the defaults elsewhere.
void load_params(const char* path, ClassParams (&params)[kClasses]) {
  for (int c = 0; c < kClasses; ++c) params[c] = kDefault;
  if (!path) return;
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const TuneEntry& e : read_cache(path)) {
    if (e.arch != arch || e.op != "batched" || e.dtype != "f32") continue;
    for (int c = 0; c < kClasses; ++c) {
      const int64_t lo = c == 0 ? 1 : kClassHi[c - 1] + 1;
      if (e.lo == lo && e.hi == kClassHi[c] && (e.gram_tile == 64 || e.gram_tile == 128) &&
          solve_slot(e.solve_threads) >= 0 && e.solve_per_cu >= 0)
        params[c] = ClassParams{e.gram_tile, e.solve_threads, e.solve_per_cu};
    }
  }
}

// ---- launches shared by the plan and the tuner ---------------------------------------------
struct BatchBuffers {
  const BatchDesc* desc;
  const float *A_pool, *B_pool;
  float *Q_pool, *q_pool, *X_pool, *vec_pool;
  double* s_pool;
  int32_t *iters, *status;
  double* kkt;
  int64_t* rows_read;
};

// The Gram launches of a list of items laid out as diag64 | diag128 | off64 | off128.
hipError_t launch_gram_lists(const BatchGramItem* items, const int64_t (&cnt)[4],
                             const BatchBuffers& b, hipStream_t st) {
  int64_t off = 0;
  hipError_t e = hipSuccess;
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    const int bm = (l & 1) ? 128 : 64;
    const bool diag = l < 2;
    e = nnls::launch_batched_gram(bm, diag, items + off, cnt[l], b.desc, b.A_pool, b.B_pool,
                                  b.Q_pool, b.q_pool, b.s_pool, st);
    off += cnt[l];
  }
  return e;
}

const void* solve_kernel(int slot) {
  switch (slot) {
    case 0: return (const void*)nnls::batched_solve_kernel<256>;
    case 1: return (const void*)nnls::batched_solve_kernel<512>;
    default: return (const void*)nnls::batched_solve_kernel<1024>;
  }
}

// Dynamic LDS and resident grid of the solver class `slot` for problems up to max_n, with at
// most per_cu_cap workgroups per compute unit (0: as many as fit).
hipError_t solve_launch_shape(int slot, int64_t max_n, int64_t count, int per_cu_cap,
                              size_t& lds, int64_t& grid) {
  const int nt = nnls::kSolveThreads[slot];
  lds = nnls::sw_lds_layout(max_n, sizeof(float), nt).total;
  int dev = 0, cus = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipError_t e = hipFuncSetAttribute(solve_kernel(slot),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, solve_kernel(slot), nt, lds);
  if (e != hipSuccess) return e;
  per_cu = std::max(per_cu, 1);
  if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
  grid = std::min<int64_t>(count, (int64_t)cus * per_cu);
  return hipSuccess;
}

hipError_t launch_solve_class(int slot, const nnls::BatchSolveArgs& B, size_t lds, int64_t grid,
                              hipStream_t st) {
  if (B.count <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), blk((unsigned)nnls::kSolveThreads[slot]);
  switch (slot) {
    case 0: hipLaunchKernelGGL(nnls::batched_solve_kernel<256>, g, blk, lds, st, B); break;
    case 1: hipLaunchKernelGGL(nnls::batched_solve_kernel<512>, g, blk, lds, st, B); break;
    default: hipLaunchKernelGGL(nnls::batched_solve_kernel<1024>, g, blk, lds, st, B); break;
  }
  return hipGetLastError();
}

nnls::BatchSolveArgs solve_args(const BatchBuffers& b, const BatchDesc* desc, const int* order,
                                int64_t count, int* counter, double tol, int max_iter) {
  nnls::BatchSolveArgs B;
  B.desc = desc;
  B.order = order;
  B.count = count;
  B.counter = counter;
  B.Q_pool = b.Q_pool;
  B.q_pool = b.q_pool;
  B.s_pool = b.s_pool;
  B.X_pool = b.X_pool;
  B.vec_pool = b.vec_pool;
  B.tol = tol;
  B.max_iter = max_iter;
  B.iters = b.iters;
  B.kkt = b.kkt;
  B.status = b.status;
  B.rows_read = b.rows_read;
  return B;
}

}  // namespace

extern "C" {

size_t nnls_batched_workspace_bytes(const nnls_problem_desc* host_desc, int64_t count) {
  if (!host_desc || count < 1) return 0;
  int64_t sum_n = 0, items = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t n = host_desc[i].n > 0 ? host_desc[i].n : 0;
    sum_n += n;
    items += item_bound(n);
  }
  return plan_layout(count, sum_n, items).total;
}

int nnls_batched_plan_create(const nnls_problem_desc* host_desc, int64_t count, double tol,
                             int32_t max_iter, const char* tune_cache, const float* A_pool,
                             const float* B_pool, float* Q_pool, float* q_pool, double* s_pool,
                             float* X_pool, int32_t* iters, double* kkt, int32_t* status,
                             int64_t* rows_read, void* ws, size_t ws_bytes, void* capture_stream,
                             nnls_plan** out) {
  if (!out) return NNLS_E_ARG;
  *out = nullptr;
  if (!capture_stream) return NNLS_E_ARG;  // the null stream cannot be captured
  if (!host_desc || count < 1 || count > (1 << 30)) return NNLS_E_ARG;
  if (!A_pool || !B_pool || !Q_pool || !q_pool || !s_pool || !X_pool || !iters || !kkt ||
      !status)
    return NNLS_E_ARG;
  if (!(tol >= 0.0) || max_iter < 0) return NNLS_E_ARG;
  int64_t sum_n = 0, max_items = 0;
  for (int64_t i = 0; i < count; ++i) {
    const nnls_problem_desc& p = host_desc[i];
    if (p.d < 1 || p.n < 1 || p.offA < 0 || p.offB < 0 || p.offQ < 0 || p.offq < 0 || p.offX < 0)
      return NNLS_E_ARG;
    if (p.n > nnls::BATCH_MAX_N) return NNLS_E_UNSUPPORTED;
    if (p.d > (1 << 30)) return NNLS_E_UNSUPPORTED;
    sum_n += p.n;
    max_items += item_bound(p.n);
  }
  const PlanLayout L = plan_layout(count, sum_n, max_items);
  if (!ws || ws_bytes < L.total) return NNLS_E_WORKSPACE;

  ClassParams params[kClasses];
  load_params(tune_cache, params);

  // descriptors, Gram items (diag64 | diag128 | off64 | off128, each longest d first) and the
  // longest-first order of each solver class
  std::vector<BatchDesc> dd(count);
  std::vector<BatchGramItem> lists[4];
  std::vector<int> order[nnls::kSolveGroups];
  std::vector<double> cost(count);
  int64_t group_max_n[nnls::kSolveGroups] = {};
  for (int64_t i = 0; i < count; ++i) {
    const nnls_problem_desc& p = host_desc[i];
    dd[i] = BatchDesc{p.d, p.n, p.offA, p.offB, p.offQ, p.offq, p.offX, 0};
    cost[i] = problem_cost(p.d, p.n);
    const ClassParams& cp = params[size_class(p.n)];
    const int li = cp.gram_tile == 128 ? 1 : 0;
    problem_items((int32_t)i, p.n, cp.gram_tile, lists[li], lists[2 + li]);
    const int grp = solve_slot(cp.solve_threads) * nnls::kCaps + cap_index(cp.solve_per_cu);
    order[grp].push_back((int)i);
    group_max_n[grp] = std::max<int64_t>(group_max_n[grp], p.n);
  }
  std::vector<BatchGramItem> items;
  int64_t cnt[4];
  for (int l = 0; l < 4; ++l) {
    std::stable_sort(lists[l].begin(), lists[l].end(),
                     [&](const BatchGramItem& a, const BatchGramItem& b) {
                       return dd[a.p].d > dd[b.p].d;
                     });
    cnt[l] = (int64_t)lists[l].size();
    items.insert(items.end(), lists[l].begin(), lists[l].end());
  }
  std::vector<int> orders;
  int64_t order_off[nnls::kSolveGroups];
  for (int c = 0; c < nnls::kSolveGroups; ++c) {
    std::stable_sort(order[c].begin(), order[c].end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
    order_off[c] = (int64_t)orders.size();
    orders.insert(orders.end(), order[c].begin(), order[c].end());
  }

  char* base = (char*)ws;
  hipStream_t st = (hipStream_t)capture_stream;
  // one-time setup copies (blocking: the host vectors are released on return)
  hipError_t e = hipMemcpy(base + L.desc, dd.data(), sizeof(BatchDesc) * count,
                           hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(base + L.items, items.data(), sizeof(BatchGramItem) * items.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + L.order, orders.data(), sizeof(int) * count, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }

  BatchBuffers bb{(const BatchDesc*)(base + L.desc), A_pool, B_pool, Q_pool, q_pool, X_pool,
                  (float*)(base + L.vec), s_pool, iters, status, kkt, rows_read};
  int* counters = (int*)(base + L.counter);
  nnls::BatchSolveArgs args[nnls::kSolveGroups];
  size_t lds[nnls::kSolveGroups] = {};
  int64_t grid[nnls::kSolveGroups] = {};
  for (int c = 0; c < nnls::kSolveGroups && e == hipSuccess; ++c) {
    args[c] = solve_args(bb, bb.desc, (const int*)(base + L.order) + order_off[c],
                         (int64_t)order[c].size(), counters + 64 * c, tol, max_iter);
    if (!order[c].empty())
      e = solve_launch_shape(c / nnls::kCaps, group_max_n[c], args[c].count,
                             kPerCuCaps[c % nnls::kCaps], lds[c], grid[c]);
  }
  if (e == hipSuccess) e = nnls::prepare_batched_gram();  // attributes are set outside capture
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }
  // the group with the most expensive problem goes first
  int slots[nnls::kSolveGroups];
  std::iota(slots, slots + nnls::kSolveGroups, 0);
  std::sort(slots, slots + nnls::kSolveGroups, [&](int a, int b) {
    const double ca = order[a].empty() ? -1.0 : cost[order[a][0]];
    const double cb = order[b].empty() ? -1.0 : cost[order[b][0]];
    return ca > cb;
  });

  nnls_plan* plan = new (std::nothrow) nnls_plan();
  if (!plan) return NNLS_E_HIP;
  plan->count = count;
  // The solver classes are parallel branches of the graph after the Gram: each is a resident
  // grid sized to fill the GPU, so a later class's workgroups start on the compute units the
  // earlier class frees as its queue runs dry (its tail) instead of after it.  The side
  // streams and events only carry the capture (default priority; released below).
  hipStream_t side[nnls::kSolveGroups] = {};
  hipEvent_t fork = nullptr, join[nnls::kSolveGroups] = {};
  e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int i = 1; i < nnls::kSolveGroups && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(nnls::batched_queue_reset, dim3(1), dim3(64), 0, st, counters,
                       nnls::kSolveGroups);
    hipError_t e1 = launch_gram_lists((const BatchGramItem*)(base + L.items), cnt, bb, st);
    if (e1 == hipSuccess) e1 = hipEventRecord(fork, st);
    for (int i = 0; i < nnls::kSolveGroups && e1 == hipSuccess; ++i) {
      const int g = slots[i];
      if (args[g].count <= 0) continue;
      hipStream_t s_i = i == 0 ? st : side[i];
      if (i > 0) e1 = hipStreamWaitEvent(s_i, fork, 0);
      if (e1 == hipSuccess)
        e1 = launch_solve_class(g / nnls::kCaps, args[g], lds[g], grid[g], s_i);
      if (e1 == hipSuccess && i > 0) e1 = hipEventRecord(join[i], s_i);
      if (e1 == hipSuccess && i > 0) e1 = hipStreamWaitEvent(st, join[i], 0);
    }
    hipError_t e2 = hipGetLastError();
    e = hipStreamEndCapture(st, &plan->graph);
    if (e == hipSuccess && e1 != hipSuccess) e = e1;
    if (e == hipSuccess && e2 != hipSuccess) e = e2;
  }
  for (int i = 1; i < nnls::kSolveGroups; ++i) {
    if (join[i]) (void)hipEventDestroy(join[i]);
    if (side[i]) (void)hipStreamDestroy(side[i]);
  }
  if (fork) (void)hipEventDestroy(fork);
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

int nnls_autotune(const char* cache_path, int op, const int64_t* shapes, int64_t count,
                  void* stream) {
  if (!cache_path || !shapes || count < 1 || count > (1 << 24)) return NNLS_E_ARG;
  if (op != NNLS_TUNE_BATCHED) return NNLS_E_ARG;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t d = shapes[2 * i], n = shapes[2 * i + 1];
    if (d < 1 || n < 1) return NNLS_E_ARG;
    if (n > nnls::BATCH_MAX_N || d > 16384) return NNLS_E_UNSUPPORTED;
  }
  const std::string arch = device_arch();
  if (arch.empty()) return NNLS_E_HIP;
  hipStream_t st = (hipStream_t)stream;
  constexpr int64_t kPerClass = 1024;  // problems measured per size class
  constexpr int kReps = 3;

  // shapes of each class, thinned evenly to at most kPerClass
  std::vector<std::pair<int64_t, int64_t>> by_class[kClasses];
  for (int64_t i = 0; i < count; ++i)
    by_class[size_class(shapes[2 * i + 1])].push_back({shapes[2 * i], shapes[2 * i + 1]});
  std::vector<TuneEntry> fresh;
  hipError_t e = hipSuccess;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (e == hipSuccess) e = nnls::prepare_batched_gram();
  for (int c = 0; c < kClasses && e == hipSuccess; ++c) {
    const auto& all = by_class[c];
    if (all.empty()) continue;
    const int64_t m = std::min<int64_t>(kPerClass, (int64_t)all.size());
    std::vector<BatchDesc> dd(m);
    int64_t offA = 0, offB = 0, offQ = 0, offq = 0, max_n = 0, items_max = 0;
    for (int64_t i = 0; i < m; ++i) {
      const auto& sh = all[(size_t)(i * (int64_t)all.size() / m)];
      dd[i] = BatchDesc{sh.first, sh.second, offA, offB, offQ, offq, offq, 0};
      offA += sh.first * sh.second;
      offB += sh.first;
      offQ += sh.second * sh.second;
      offq += sh.second;
      max_n = std::max(max_n, sh.second);
      items_max += item_bound(sh.second);
    }
    // device buffers of the measurement (a setup call: allocated here, freed below)
    const size_t bytes[] = {sizeof(BatchDesc) * m, sizeof(float) * offA, sizeof(float) * offB,
                            sizeof(float) * offQ, sizeof(float) * offq, sizeof(double) * offq,
                            sizeof(float) * offq, sizeof(float) * 3 * offq,
                            sizeof(int32_t) * m, sizeof(double) * m, sizeof(int32_t) * m,
                            sizeof(BatchGramItem) * items_max, sizeof(int) * m, sizeof(int) * 64};
    constexpr int NB = sizeof(bytes) / sizeof(bytes[0]);
    void* buf[NB] = {};
    for (int b = 0; b < NB && e == hipSuccess; ++b) e = hipMalloc(&buf[b], bytes[b]);
    if (e == hipSuccess)
      e = hipMemcpy(buf[0], dd.data(), sizeof(BatchDesc) * m, hipMemcpyHostToDevice);
    BatchBuffers bb{(const BatchDesc*)buf[0], (const float*)buf[1], (const float*)buf[2],
                    (float*)buf[3], (float*)buf[4], (float*)buf[6], (float*)buf[7],
                    (double*)buf[5], (int32_t*)buf[8], (int32_t*)buf[10], (double*)buf[9],
                    nullptr};
    if (e == hipSuccess) {
      hipLaunchKernelGGL(nnls::tune_problem_kernel, dim3((unsigned)m), dim3(256), 0, st,
                         bb.desc, (float*)buf[1], (float*)buf[2]);
      e = hipGetLastError();
    }
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      return problem_cost(dd[a].d, dd[a].n) > problem_cost(dd[b].d, dd[b].n);
    });
    if (e == hipSuccess)
      e = hipMemcpy(buf[12], ord.data(), sizeof(int) * m, hipMemcpyHostToDevice);

    auto timed = [&](auto&& body, float& ms) {
      hipError_t r = body();  // warm-up
      float best = 1e30f;
      for (int rep = 0; rep < kReps && r == hipSuccess; ++rep) {
        r = hipEventRecord(ev0, st);
        if (r == hipSuccess) r = body();
        if (r == hipSuccess) r = hipEventRecord(ev1, st);
        if (r == hipSuccess) r = hipEventSynchronize(ev1);
        float t = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&t, ev0, ev1);
        best = std::min(best, t);
      }
      ms = best;
      return r;
    };
    // Gram: each tile size over the class's problems
    float gram_ms[2] = {0.f, 0.f};
    for (int t = 0; t < 2 && e == hipSuccess; ++t) {
      const int bm = t == 0 ? 64 : 128;
      std::vector<BatchGramItem> lists[4], items;
      for (int64_t i = 0; i < m; ++i)
        problem_items((int32_t)i, dd[i].n, bm, lists[t], lists[2 + t]);
      int64_t cnt[4];
      for (int l = 0; l < 4; ++l) {
        cnt[l] = (int64_t)lists[l].size();
        items.insert(items.end(), lists[l].begin(), lists[l].end());
      }
      e = hipMemcpy(buf[11], items.data(), sizeof(BatchGramItem) * items.size(),
                    hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = timed([&]() { return launch_gram_lists((const BatchGramItem*)buf[11], cnt, bb, st); },
                  gram_ms[t]);
    }
    const int best_tile = gram_ms[0] <= gram_ms[1] ? 64 : 128;
    // the Gram of the chosen size leaves Q, q, s for the solver measurements
    if (e == hipSuccess) {
      std::vector<BatchGramItem> lists[4], items;
      const int t = best_tile == 64 ? 0 : 1;
      for (int64_t i = 0; i < m; ++i)
        problem_items((int32_t)i, dd[i].n, best_tile, lists[t], lists[2 + t]);
      int64_t cnt[4];
      for (int l = 0; l < 4; ++l) {
        cnt[l] = (int64_t)lists[l].size();
        items.insert(items.end(), lists[l].begin(), lists[l].end());
      }
      e = hipMemcpy(buf[11], items.data(), sizeof(BatchGramItem) * items.size(),
                    hipMemcpyHostToDevice);
      if (e == hipSuccess) e = launch_gram_lists((const BatchGramItem*)buf[11], cnt, bb, st);
    }
    // solver: each workgroup size, with as many resident workgroups as fit and with one per
    // compute unit, over the class's problems (tolerance and cap of the batched workload)
    float solve_ms[nnls::kSolveGroups] = {};
    for (int g = 0; g < nnls::kSolveGroups && e == hipSuccess; ++g) {
      const int slot = g / nnls::kCaps;
      size_t lds = 0;
      int64_t grid = 0;
      e = solve_launch_shape(slot, max_n, m, kPerCuCaps[g % nnls::kCaps], lds, grid);
      const nnls::BatchSolveArgs B =
          solve_args(bb, bb.desc, (const int*)buf[12], m, (int*)buf[13], 5e-6, 20000);
      if (e == hipSuccess)
        e = timed(
            [&]() {
              hipLaunchKernelGGL(nnls::batched_queue_reset, dim3(1), dim3(64), 0, st,
                                 (int*)buf[13], 1);
              return launch_solve_class(slot, B, lds, grid, st);
            },
            solve_ms[g]);
    }
    for (int b = 0; b < NB; ++b)
      if (buf[b]) (void)hipFree(buf[b]);
    if (e != hipSuccess) break;
    int best = 0;
    for (int g = 1; g < nnls::kSolveGroups; ++g)
      if (solve_ms[g] < solve_ms[best]) best = g;
    TuneEntry te;
    te.arch = arch;
    te.op = "batched";
    te.dtype = "f32";
    te.lo = c == 0 ? 1 : kClassHi[c - 1] + 1;
    te.hi = kClassHi[c];
    te.gram_tile = best_tile;
    te.solve_threads = nnls::kSolveThreads[best / nnls::kCaps];
    te.solve_per_cu = kPerCuCaps[best % nnls::kCaps];
    std::string sm;
    for (int g = 0; g < nnls::kSolveGroups; ++g) {
      char item[48];
      snprintf(item, sizeof(item), "%s\"%d%s\": %.4f", g ? ", " : "",
               nnls::kSolveThreads[g / nnls::kCaps], kPerCuCaps[g % nnls::kCaps] ? "/1" : "",
               solve_ms[g]);
      sm += item;
    }
    char line[800];
    snprintf(line, sizeof(line),
             "{\"arch\": \"%s\", \"op\": \"batched\", \"dtype\": \"f32\", \"n_lo\": %lld, "
             "\"n_hi\": %lld, \"gram_tile\": %d, \"solve_threads\": %d, \"solve_wgs_per_cu\": %d, "
             "\"problems\": %lld, \"gram_ms\": {\"64\": %.4f, \"128\": %.4f}, \"solve_ms\": {%s}}",
             arch.c_str(), (long long)te.lo, (long long)te.hi, te.gram_tile, te.solve_threads,
             te.solve_per_cu, (long long)m, gram_ms[0], gram_ms[1], sm.c_str());
    te.line = line;
    fresh.push_back(te);
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (e != hipSuccess) {
    plan_fail(e);
    return NNLS_E_HIP;
  }
  // merge with the entries already in the cache: a fresh entry replaces the one with its key
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::vector<TuneEntry> all = read_cache(cache_path);
  for (const TuneEntry& f : fresh) {
    bool replaced = false;
    for (TuneEntry& o : all)
      if (o.arch == f.arch && o.op == f.op && o.dtype == f.dtype && o.lo == f.lo && o.hi == f.hi) {
        o = f;
        replaced = true;
      }
    if (!replaced) all.push_back(f);
  }
  return write_cache(cache_path, all) ? NNLS_OK : NNLS_E_IO;
}

}  // extern "C"
