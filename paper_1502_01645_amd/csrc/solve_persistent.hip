// Algorithm 2 for one large right-hand side: a persistent cooperative kernel over the whole GPU.
//
// One update costs two grid-wide barriers:
//   phase 1  every workgroup owns a (column block, passive-row group) pair of the product
//            w = Q gbar.  Q is symmetric, so only the rows of Q in the passive set are read, each
//            row segment contiguous; the workgroup writes its partial w over its column block and
//            its share of den = gbar^T Q gbar.  Everything phase 2 needs that does not depend on
//            alpha (stop statistics, clip thresholds, the owner's own entries) is loaded here too,
//            so its latency hides behind the product.
//   -- barrier --
//   phase 2  every workgroup forms den and alpha, and the clipped set C (entries whose
//            projection hits zero: y_i / gbar_i < alpha); the owner of each 64-entry chunk sums
//            the partials of w, adds the clip correction Q[C, i] * delta_C, updates y and the
//            gradient, and publishes the next passive mask, masked gradient, clip thresholds
//            and its share of the stop statistics.
//   -- barrier --
// The stop test of an iterate is evaluated during the next phase 1; a converged gradient is
// recomputed exactly (Q y + q over the rows with y > 0) before the stop is accepted.
//
// Cross-workgroup state (y, gradient, masks, partials, statistics) is written and read with
// agent-scope relaxed atomics, which on gfx950 are sc1 accesses that bypass the per-XCD L2, so
// the barrier needs no L2 write-back or invalidate.  The barrier uses monotonic counters: one
// per group of workgroups, then one top counter, then a generation word the waiters poll.
// Q itself is read-only during the launch and uses ordinary cached loads.  The published state
// is double-buffered by iteration parity: phase 2 reads the current copy (every workgroup needs
// it for the clipped set) while owners write the next one.
#include "common.hpp"
#include "grid_sync.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int SP_NT = 512;     // threads per workgroup (8 waves)
constexpr int SP_NW = SP_NT / kWave;
constexpr int SP_CB = 1024;    // columns per block in phase 1 (4 per thread, two row halves)
constexpr int SP_CHUNK = 64;   // entries per owner chunk (one wave, one 64-bit mask word)
constexpr int SP_TPT = 32;     // clip thresholds held per thread: n <= SP_NT * SP_TPT
constexpr int64_t SP_MAX_N = (int64_t)SP_NT * SP_TPT;
constexpr size_t SP_MAX_LDS = 160 * 1024;
constexpr int SP_RPT = 4;      // row-range entries per thread in phase 1: n / R <= SP_NT * SP_RPT

struct SpArgs {
  int n, G, nb, R, nw, rows_max;
  const float* Q;
  const float* q;
  const double* s;
  const float* Y0;
  float* X;
  double tol;
  int max_iter;
  int32_t* iters;
  double* kkt;
  int32_t* status;
  int64_t* rows_read;
  float* trace;  // [trace_len][2] per-update record (r, ||gbar||^2), or nullptr
  int trace_len;
  // workspace; y, g, p, t and the masks have two copies selected by iteration parity
  float *y[2], *g[2], *p[2], *t[2];  // t: clip threshold y_i / gbar_i, +inf if i cannot clip
  uint64_t *pmask[2], *ymask[2];
  float *part, *scal;
  unsigned* bar;   // grid barrier words, with the abort word (grid_sync.hpp)
  int spin_limit;  // polls before a barrier wait gives up (never reached in a normal launch)
};

__device__ __forceinline__ float sp_block_sum(float v, float* red) {
  return block_sum<float, SP_NT>(v, red);
}

struct SpLds {
  int* rowidx;    // [rows_max]
  float* rowval;  // [rows_max]
  int* cidx;      // [n]
  float* cval;    // [n]
  float* half;    // [256 * 4] second-half partial of the row product
  float* wred;    // [SP_NW][64]
  float* cred;    // [SP_NW][64]
  float* stats;   // [8]
  float* redF;    // [SP_NW]
  int* redI;      // [SP_NW]
};

// Phase-1 product over the rows selected by `mask` with row weights vec[row].  Workgroup g is
// (column block g % nb, row group g / nb); row group r takes the selected rows whose index lies
// in [n r / R, n (r + 1) / R), so it needs only its own mask words and weights (one round of
// loads, no grid-wide scan).  Threads t and t + 256 share 4 columns and split the rows by
// parity.  The partial over the block goes to part[r, block]; returns this workgroup's share of
// dot(result, vec).
__device__ float rows_product(const SpArgs& A, const uint64_t* mask, const float* vec,
                             const SpLds& L) {
  const int g = blockIdx.x;
  const int c = g % A.nb;
  const int r = g / A.nb;
  const bool active = r < A.R;
  const int n = A.n;
  const int quad = threadIdx.x & 255;
  const int half = threadIdx.x >> 8;
  const int col = c * SP_CB + 4 * quad;
  const bool own_col = active && col < n;
  const int i_lo = active ? (int)(((int64_t)n * r) / A.R) : 0;
  const int i_hi = active ? (int)(((int64_t)n * (r + 1)) / A.R) : 0;
  const int w_lo = i_lo / 64;
  const int nwords = active ? (i_hi + 63) / 64 - w_lo : 0;
  // one round: mask words, row weights of the range, and vec over the own columns
  uint64_t* words = (uint64_t*)L.half;  // scratch until the partial reduction below
  for (int m = threadIdx.x; m < nwords; m += SP_NT) words[m] = ld_sc(mask + w_lo + m);
  const int span = i_hi - i_lo;
  float wv[SP_RPT];
#pragma unroll
  for (int u = 0; u < SP_RPT; ++u) {
    const int i = i_lo + threadIdx.x + u * SP_NT;
    wv[u] = (threadIdx.x + u * SP_NT < span) ? ld_sc(vec + i) : 0.f;
  }
  f32x4 pv = {0.f, 0.f, 0.f, 0.f};
  if (half == 0 && own_col) {
#pragma unroll
    for (int e = 0; e < 4; ++e) pv[e] = ld_sc(vec + col + e);
  }
  __syncthreads();
  int cnt = 0;
#pragma unroll
  for (int u = 0; u < SP_RPT; ++u) {
    const int off = threadIdx.x + u * SP_NT;
    const int i = i_lo + off;
    if (off < span && ((words[i / 64 - w_lo] >> (i & 63)) & 1ull)) ++cnt;
  }
  int total;
  int pos = block_exclusive_scan<SP_NT>(cnt, L.redI, total);
#pragma unroll
  for (int u = 0; u < SP_RPT; ++u) {
    const int off = threadIdx.x + u * SP_NT;
    const int i = i_lo + off;
    if (off < span && ((words[i / 64 - w_lo] >> (i & 63)) & 1ull)) {
      L.rowidx[pos] = i;
      L.rowval[pos] = wv[u];
      ++pos;
    }
  }
  __syncthreads();
  const int cnt_rows = total;

  float dot = 0.f;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (own_col) {
    const float* Qc = A.Q + col;
    int k = half;
    for (; k + 30 < cnt_rows; k += 32) {
      f32x4 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = *(const f32x4*)(Qc + (int64_t)L.rowidx[k + 2 * u] * n);
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += L.rowval[k + 2 * u] * v[u];
    }
    for (; k + 6 < cnt_rows; k += 8) {
      f32x4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = *(const f32x4*)(Qc + (int64_t)L.rowidx[k + 2 * u] * n);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += L.rowval[k + 2 * u] * v[u];
    }
    for (; k < cnt_rows; k += 2) acc += L.rowval[k] * *(const f32x4*)(Qc + (int64_t)L.rowidx[k] * n);
  }
  if (half == 1) *(f32x4*)(L.half + 4 * quad) = acc;
  __syncthreads();
  if (half == 0 && own_col) {
    acc += *(const f32x4*)(L.half + 4 * quad);
    float* dst = A.part + (int64_t)r * n + col;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      st_sc(dst + e, acc[e]);
      dot += acc[e] * pv[e];
    }
  }
  return sp_block_sum(dot, L.redF);
}

// Owner update of one 64-entry chunk by wave 0: publishes y, gradient, masked gradient, clip
// threshold and mask words into copy `dst`, and adds the chunk's statistics to stats[0..3]
// (sum of gbar^2, sum of min(y, grad)^2, passive count, non-finite count, count of y > 0).
__device__ __forceinline__ void publish_entry(const SpArgs& A, int dst, int i, bool valid,
                                              float yi, float gi, int chunk, float* stats) {
  const bool pas = valid && ((yi > 0.f) || (gi < 0.f));
  const float pi = pas ? gi : 0.f;
  const bool cand = pas && (pi > 0.f) && (yi > 0.f);
  const uint64_t pm = __ballot(pas);
  const uint64_t ym = __ballot(valid && yi > 0.f);
  if (valid) {
    st_sc(A.y[dst] + i, yi);
    st_sc(A.g[dst] + i, gi);
    st_sc(A.p[dst] + i, pi);
    st_sc(A.t[dst] + i, cand ? yi / pi : __builtin_inff());
  }
  if ((threadIdx.x & 63) == 0) {
    st_sc(A.pmask[dst] + chunk, pm);
    st_sc(A.ymask[dst] + chunk, ym);
  }
  const float m = yi < gi ? yi : gi;
  const bool bad = valid && (!__builtin_isfinite(yi) || !__builtin_isfinite(gi));
  const float s_num = wave_sum(valid ? pi * pi : 0.f);
  const float s_res = wave_sum(valid ? m * m : 0.f);
  const float s_cnt = wave_sum(pas ? 1.f : 0.f);
  const float s_bad = wave_sum(bad ? 1.f : 0.f);
  const float s_pos = wave_sum((valid && yi > 0.f) ? 1.f : 0.f);
  if ((threadIdx.x & 63) == 0) {
    stats[0] += s_num;
    stats[1] += s_res;
    stats[2] += s_cnt;
    stats[3] += s_bad;
    stats[4] += s_pos;
  }
}

// Sum over row groups of the phase-1 partials at entry i for the groups r = wave (mod 8).
__device__ __forceinline__ float partial_sum(const SpArgs& A, int i, int wave) {
  float s = 0.f;
  int r = wave;
  for (; r + 7 * SP_NW < A.R; r += 8 * SP_NW) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ld_sc(A.part + (int64_t)(r + u * SP_NW) * A.n + i);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; r < A.R; r += SP_NW) s += ld_sc(A.part + (int64_t)r * A.n + i);
  return s;
}

__device__ __forceinline__ void publish_stats(const SpArgs& A, const SpLds& L) {
  __syncthreads();
  if (threadIdx.x < 5) st_sc(A.scal + blockIdx.x * 8 + 1 + threadIdx.x, L.stats[threadIdx.x]);
}

__global__ __launch_bounds__(SP_NT) void solve_persistent_kernel(SpArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  SpLds L;
  {
    unsigned char* p = smem;
    auto take = [&](size_t bytes) {
      unsigned char* r = p;
      p += (bytes + 15) & ~(size_t)15;
      return (void*)r;
    };
    L.rowidx = (int*)take(sizeof(int) * A.rows_max);
    L.rowval = (float*)take(sizeof(float) * A.rows_max);
    L.cidx = (int*)take(sizeof(int) * A.n);
    L.cval = (float*)take(sizeof(float) * A.n);
    L.half = (float*)take(sizeof(float) * 1024);
    L.wred = (float*)take(sizeof(float) * SP_NW * 64);
    L.cred = (float*)take(sizeof(float) * SP_NW * 64);
    L.stats = (float*)take(sizeof(float) * 8);
    L.redF = (float*)take(sizeof(float) * SP_NW);
    L.redI = (int*)take(sizeof(int) * SP_NW);
  }

  const int n = A.n, G = A.G;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // each workgroup owns at most one 64-entry chunk (n <= 64 G is required on the host)
  const int chunk = blockIdx.x;
  const bool owner = chunk < A.nw;
  const int oi = chunk * SP_CHUNK + lane;  // owned entry of this lane (wave 0)
  const bool ovalid = owner && oi < n;
  unsigned epoch = 0;

  // ---- start point: y = max(Y0, 0) or 0, gradient = q (refreshed first for a warm start)
  if (threadIdx.x < 8) L.stats[threadIdx.x] = 0.f;
  __syncthreads();
  if (owner && wave == 0) {
    float yi = 0.f, gi = 0.f;
    if (ovalid) {
      gi = A.q[oi];
      if (A.Y0) {
        yi = A.Y0[oi];
        yi = yi > 0.f ? yi : 0.f;
      }
    }
    publish_entry(A, 0, oi, ovalid, yi, gi, chunk, L.stats);
  }
  publish_stats(A, L);
  float qn2;
  {
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += SP_NT) acc += A.q[i] * A.q[i];
    qn2 = sp_block_sum(acc, L.redF);
  }
  const double qscale = qn2 > 0.f ? sqrt((double)qn2) : 1.0;
  // a barrier that gave up (every workgroup leaves at its next wait) ends the solve
  bool timed_out = !grid_barrier(A.bar, G, epoch, A.spin_limit);

  int cur = 0;
  int it = 0;
  int64_t rows = 0;  // rows of Q read by the products
  bool fresh = (A.Y0 == nullptr);
  bool need_refresh = (A.Y0 != nullptr);
  int status = NNLS_MAXITER_DEV;
  double r_now = 0.0;

  while (!timed_out) {
    if (need_refresh) {
      // gradient = Q y + q over the rows with y > 0
      {
        const float v = (threadIdx.x < G) ? ld_sc(A.scal + threadIdx.x * 8 + 5) : 0.f;
        rows += (int64_t)sp_block_sum(v, L.redF);
      }
      rows_product(A, A.ymask[cur], A.y[cur], L);
      if (!grid_barrier(A.bar, G, epoch, A.spin_limit)) {
        timed_out = true;
        break;
      }
      if (threadIdx.x < 8) L.stats[threadIdx.x] = 0.f;
      __syncthreads();
      if (owner) {
        L.wred[wave * 64 + lane] = (oi < n) ? partial_sum(A, oi, wave) : 0.f;
        __syncthreads();
        if (wave == 0) {
          float w = 0.f;
#pragma unroll
          for (int v = 0; v < SP_NW; ++v) w += L.wred[v * 64 + lane];
          const float yi = ovalid ? ld_sc(A.y[cur] + oi) : 0.f;
          const float gi = ovalid ? A.q[oi] + w : 0.f;
          publish_entry(A, cur ^ 1, oi, ovalid, yi, gi, chunk, L.stats);
        }
      }
      publish_stats(A, L);
      if (!grid_barrier(A.bar, G, epoch, A.spin_limit)) {
        timed_out = true;
        break;
      }
      cur ^= 1;
      need_refresh = false;
      fresh = true;
    }

    // ---- phase 1.  Loads that do not depend on alpha go first.
    float sv[4] = {0.f, 0.f, 0.f, 0.f};
    if (threadIdx.x < G) {
#pragma unroll
      for (int u = 0; u < 4; ++u) sv[u] = ld_sc(A.scal + threadIdx.x * 8 + 1 + u);
    }
    // thresholds of entries threadIdx.x + u * SP_NT (coalesced across the wave)
    float tv[SP_TPT];
#pragma unroll
    for (int u = 0; u < SP_TPT; ++u) {
      const int j = threadIdx.x + u * SP_NT;
      tv[u] = (j < n) ? ld_sc(A.t[cur] + j) : __builtin_inff();
    }
    float y0 = 0.f, g0 = 0.f, p0 = 0.f;
    if (ovalid && wave == 0) {
      y0 = ld_sc(A.y[cur] + oi);
      g0 = ld_sc(A.g[cur] + oi);
      p0 = ld_sc(A.p[cur] + oi);
    }
    const float den_part = rows_product(A, A.pmask[cur], A.p[cur], L);
    if (threadIdx.x == 0) st_sc(A.scal + blockIdx.x * 8 + 0, den_part);

    // stop test of the current iterate (identical in every workgroup): one four-wide
    // reduction of the published statistics
    float num, res, npass, bad;
    {
#pragma unroll
      for (int u = 0; u < 4; ++u) sv[u] = wave_sum(sv[u]);
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) L.wred[u * SP_NW + wave] = sv[u];
      }
      __syncthreads();
      float tot[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < SP_NW; ++v) tot[u] += L.wred[u * SP_NW + v];
      __syncthreads();
      num = tot[0];
      res = tot[1];
      npass = tot[2];
      bad = tot[3];
    }
    if (bad > 0.f) {
      status = NNLS_NONFINITE_DEV;
      break;
    }
    r_now = sqrt((double)res) / qscale;
    if (A.trace != nullptr && blockIdx.x == 0 && threadIdx.x == 0 && it < A.trace_len) {
      A.trace[2 * it] = (float)r_now;
      A.trace[2 * it + 1] = num;
    }
    if (npass == 0.f || r_now <= A.tol) {
      if (fresh) {
        status = NNLS_CONVERGED_DEV;
        break;
      }
      need_refresh = true;
      continue;
    }
    if (it >= A.max_iter) {
      if (!fresh) {
        need_refresh = true;
        continue;
      }
      status = NNLS_MAXITER_DEV;
      break;
    }
    rows += (int64_t)npass;
    if (!grid_barrier(A.bar, G, epoch, A.spin_limit)) {
      timed_out = true;
      break;
    }

    // ---- phase 2
    float dv = (threadIdx.x < G) ? ld_sc(A.scal + threadIdx.x * 8 + 0) : 0.f;
    float wsum = 0.f;
    if (owner) wsum = (oi < n) ? partial_sum(A, oi, wave) : 0.f;
    const float den = sp_block_sum(dv, L.redF);
    if (!(den > 0.f) || !__builtin_isfinite(den)) {
      status = NNLS_BREAKDOWN_DEV;
      break;
    }
    const float alpha = num / den;

    // clipped set (thread-major order): entries with threshold < alpha
    int ccount;
    {
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < SP_TPT; ++u) cnt += (tv[u] < alpha);
      int pos = block_exclusive_scan<SP_NT>(cnt, L.redI, ccount);
#pragma unroll
      for (int u = 0; u < SP_TPT; ++u) {
        if (tv[u] < alpha) {
          L.cidx[pos] = threadIdx.x + u * SP_NT;
          ++pos;
        }
      }
      __syncthreads();
      for (int m = threadIdx.x; m < ccount; m += SP_NT) {
        const int j = L.cidx[m];
        L.cval[m] = alpha * ld_sc(A.p[cur] + j) - ld_sc(A.y[cur] + j);  // delta_j
      }
      __syncthreads();
    }
    rows += ccount;

    if (threadIdx.x < 8) L.stats[threadIdx.x] = 0.f;
    if (owner) {
      float csum = 0.f;
      if (oi < n) {
        int m = wave;
        for (; m + 3 * SP_NW < ccount; m += 4 * SP_NW) {
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = A.Q[(int64_t)L.cidx[m + u * SP_NW] * n + oi];
#pragma unroll
          for (int u = 0; u < 4; ++u) csum += L.cval[m + u * SP_NW] * v[u];
        }
        for (; m < ccount; m += SP_NW) csum += L.cval[m] * A.Q[(int64_t)L.cidx[m] * n + oi];
      }
      L.wred[wave * 64 + lane] = wsum;
      L.cred[wave * 64 + lane] = csum;
      __syncthreads();
      if (wave == 0) {
        float w = 0.f, corr = 0.f;
#pragma unroll
        for (int v = 0; v < SP_NW; ++v) {
          w += L.wred[v * 64 + lane];
          corr += L.cred[v * 64 + lane];
        }
        float yi = 0.f, gi = 0.f;
        if (ovalid) {
          const float v = y0 - alpha * p0;
          yi = v > 0.f ? v : 0.f;
          gi = g0 - alpha * w + corr;
        }
        publish_entry(A, cur ^ 1, oi, ovalid, yi, gi, chunk, L.stats);
      }
    }
    publish_stats(A, L);
    if (!grid_barrier(A.bar, G, epoch, A.spin_limit)) {
      timed_out = true;
      break;
    }
    cur ^= 1;
    ++it;
    fresh = false;
  }

  // ---- outputs
  if (ovalid && wave == 0) {
    const float yi = ld_sc(A.y[cur] + oi);
    A.X[oi] = A.s ? (float)((double)yi / A.s[oi]) : yi;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.iters[0] = timed_out ? -1 : it;
    A.kkt[0] = (status == NNLS_NONFINITE_DEV || timed_out) ? __builtin_nan("") : r_now;
    A.status[0] = timed_out ? NNLS_BREAKDOWN_DEV : status;
    if (A.rows_read) A.rows_read[0] = rows;
  }
}

__global__ void grid_barrier_init_kernel(unsigned* bar) {
  for (int i = threadIdx.x; i < GS_BAR_WORDS; i += blockDim.x) bar[i] = 0u;
}

// ---- host side ------------------------------------------------------------------------------
struct SpPlan {
  int G, nb, R, nw, rows_max;
  size_t lds;
};

static int sp_device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

static SpPlan sp_plan(int64_t n, int cus) {
  SpPlan P;
  P.G = cus > 0 ? cus : 256;
  P.nb = (int)((n + SP_CB - 1) / SP_CB);
  if (P.nb > P.G) P.nb = P.G;
  P.R = P.G / P.nb;
  P.nw = (int)((n + SP_CHUNK - 1) / SP_CHUNK);
  P.rows_max = (int)((n + P.R - 1) / P.R) + 1;
  auto a16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
  P.lds = a16(sizeof(int) * P.rows_max) + a16(sizeof(float) * P.rows_max) +
          a16(sizeof(int) * n) + a16(sizeof(float) * n) + a16(sizeof(float) * 1024) +
          2 * a16(sizeof(float) * SP_NW * 64) + a16(sizeof(float) * 8) +
          a16(sizeof(float) * SP_NW) + a16(sizeof(int) * SP_NW);
  return P;
}

bool solve_persistent_supported(int64_t n, int64_t k) {
  if (k != 1 || n < 1 || n > SP_MAX_N || (n % 4) != 0) return false;
  const SpPlan P = sp_plan(n, sp_device_cus());
  return n <= (int64_t)SP_CHUNK * P.G && P.lds <= SP_MAX_LDS &&
         (n + P.R - 1) / P.R <= (int64_t)SP_NT * SP_RPT;
}

size_t solve_persistent_ws_bytes(int64_t n) {
  const SpPlan P = sp_plan(n, sp_device_cus());
  size_t b = 0;
  b += 2 * (4 * (sizeof(float) * n + 256));       // y, g, p, t (two copies)
  b += 2 * (2 * (sizeof(uint64_t) * P.nw + 256)); // masks (two copies)
  b += sizeof(float) * (size_t)P.R * n + 256;     // partials
  b += sizeof(float) * 8 * P.G + 256;             // per-workgroup scalars
  b += sizeof(unsigned) * GS_BAR_WORDS + 256;     // barrier words
  return b + 1024;
}

hipError_t launch_solve_persistent(int64_t n, const float* Q, const float* q, const double* s,
                                   double tol, int max_iter, const float* Y0, float* X,
                                   int32_t* iters, double* kkt, int32_t* status,
                                   int64_t* rows_read, float* trace, int trace_len, void* ws,
                                   hipStream_t st) {
  const SpPlan P = sp_plan(n, sp_device_cus());
  SpArgs A;
  A.n = (int)n;
  A.G = P.G;
  A.nb = P.nb;
  A.R = P.R;
  A.nw = P.nw;
  A.rows_max = P.rows_max;
  A.Q = Q;
  A.q = q;
  A.s = s;
  A.Y0 = Y0;
  A.X = X;
  A.tol = tol;
  A.max_iter = max_iter;
  A.iters = iters;
  A.kkt = kkt;
  A.status = status;
  A.rows_read = rows_read;
  A.trace = trace;
  A.trace_len = trace_len;
  A.spin_limit = spin_limit_setting();
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return (void*)r;
  };
  A.bar = (unsigned*)take(sizeof(unsigned) * GS_BAR_WORDS);
  for (int b = 0; b < 2; ++b) {
    A.y[b] = (float*)take(sizeof(float) * n);
    A.g[b] = (float*)take(sizeof(float) * n);
    A.p[b] = (float*)take(sizeof(float) * n);
    A.t[b] = (float*)take(sizeof(float) * n);
    A.pmask[b] = (uint64_t*)take(sizeof(uint64_t) * P.nw);
    A.ymask[b] = (uint64_t*)take(sizeof(uint64_t) * P.nw);
  }
  A.part = (float*)take(sizeof(float) * (size_t)P.R * n);
  A.scal = (float*)take(sizeof(float) * 8 * P.G);

  hipError_t e = hipFuncSetAttribute((const void*)solve_persistent_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)solve_persistent_kernel,
                                                   SP_NT, P.lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(grid_barrier_init_kernel, dim3(1), dim3(256), 0, st, A.bar);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {&A};
  return hipLaunchCooperativeKernel((const void*)solve_persistent_kernel, dim3(P.G), dim3(SP_NT),
                                    args, P.lds, st);
}

}  // namespace nnls
