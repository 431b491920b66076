// Algorithm 2 for one large right-hand side: a persistent cooperative kernel over the whole GPU.
//
// One update costs two grid-wide barriers:
//   phase 1  every workgroup owns a (column block, passive-row group) pair of the product
//            w = Q gbar.  Q is symmetric, so only the rows of Q in the passive set are read, each
//            row segment contiguous; the workgroup writes its partial w over its column block and
//            its share of den = gbar^T Q gbar.
//   -- barrier --
//   phase 2  every workgroup forms den and alpha, and the clipped set C (entries whose
//            projection hits zero, known from per-entry thresholds y_i / gbar_i); the owner of each
//            64-entry chunk sums the partials of w, adds the clip correction Q[C, i] * delta_C,
//            updates y and the gradient, and publishes the next passive mask, masked gradient,
//            clip thresholds and its share of the stop statistics.
//   -- barrier --
// The gradient of a converged iterate is recomputed exactly (Q y + q over rows with y > 0)
// before the stop is accepted.
//
// Cross-workgroup state (y, gradient, masks, partials, statistics) is written and read with
// agent-scope relaxed atomics, which on gfx950 are sc1 accesses that bypass the per-XCD L2, so
// the barrier needs no L2 write-back or invalidate.  The barrier uses monotonic counters: one
// per group of workgroups, then one top counter, then a generation word the waiters poll.
// Q itself is read-only during the launch and uses ordinary cached loads.  The published state
// is double-buffered by iteration parity: phase 2 reads the current copy (every workgroup needs
// it for the clipped set) while owners write the next one.
#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int SP_NT = 256;     // threads per workgroup
constexpr int SP_CB = 1024;    // columns per block in phase 1 (4 per thread)
constexpr int SP_CHUNK = 64;   // entries per owner chunk (one wave, one 64-bit mask word)
constexpr int SP_GROUPS = 8;   // barrier arrival groups
constexpr int SP_BAR_WORDS = 1024;
constexpr int SP_TPT = 64;     // clip thresholds held per thread: n <= SP_NT * SP_TPT

__device__ __forceinline__ float ld_sc(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sc(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_sc(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sc(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct SpArgs {
  int n, G, nb, R, nw, cmax, rows_max;
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
  // workspace; y, g, p, t and the masks have two copies selected by iteration parity
  float *y[2], *g[2], *p[2], *t[2];  // t: clip threshold y_i / gbar_i, +inf if i cannot clip
  uint64_t *pmask[2], *ymask[2];
  float *part, *scal;
  unsigned* bar;
};

// Grid barrier.  Every wave first waits for its own sc1 stores, so once all workgroups have
// arrived their published data is visible at the coherence point.  Counters only grow, so no
// reset can race with a later arrival; epoch is this workgroup's count of barriers passed.
__device__ __forceinline__ void grid_barrier(unsigned* bar, int G, unsigned& epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int ngroups = G < SP_GROUPS ? G : SP_GROUPS;
    const int grp = blockIdx.x % ngroups;
    const unsigned gsize = (unsigned)(G / ngroups + (grp < G % ngroups ? 1 : 0));
    unsigned* gen = bar;
    unsigned* top = bar + 32;
    unsigned* gc = bar + 64 + 32 * grp;
    const unsigned target = epoch + 1;
    const unsigned a = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a == gsize * target - 1) {
      const unsigned b =
          __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (b == (unsigned)ngroups * target - 1)
        __hip_atomic_store(gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
      __builtin_amdgcn_s_sleep(1);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  epoch += 1;
  __syncthreads();
}

// Sum of one float per thread over the workgroup (two barriers).
__device__ __forceinline__ float sp_block_sum(float v, float* red) {
  return block_sum<float, SP_NT>(v, red);
}

// Compacted positions [lo, hi) of the set bits of mask[0..nw) in index order, written to
// idx[0..hi-lo).  Each thread scans a contiguous run of words.  Returns the total bit count.
__device__ int select_bits(const uint64_t* mask, int nw, int lo, int hi, int* idx, int* redI) {
  const int per = (nw + SP_NT - 1) / SP_NT;
  const int w0 = threadIdx.x * per;
  const int w1 = w0 + per < nw ? w0 + per : nw;
  int cnt = 0;
  for (int m = w0; m < w1; ++m) cnt += __popcll(ld_sc(mask + m));
  int total;
  int pos = block_exclusive_scan<SP_NT>(cnt, redI, total);
  for (int m = w0; m < w1 && pos < hi; ++m) {
    uint64_t bits = ld_sc(mask + m);
    while (bits) {
      const int b = __ffsll((long long)bits) - 1;
      bits &= bits - 1;
      if (pos >= lo && pos < hi) idx[pos - lo] = m * 64 + b;
      ++pos;
    }
  }
  __syncthreads();
  return total;
}

// Phase-1 product over the rows selected by `mask` with row weights vec[row]: this workgroup's
// rows are the compacted range of its row group; the partial over its column block goes to
// part[r, block].  Returns this workgroup's share of dot(result, vec_block) (only meaningful
// for the line-search product, where vec = gbar).
__device__ float rows_product(const SpArgs& A, const uint64_t* mask, const float* vec,
                             int* rowidx, float* rowval, int* redI, float* redF, int& nrows) {
  const int g = blockIdx.x;
  const int c = g % A.nb;
  const int r = g / A.nb;
  const bool active = r < A.R;
  // every workgroup joins the scan (it contains barriers)
  int total = 0;
  int lo = 0, hi = 0;
  {
    // first pass: total count to derive this group's range
    const int per = (A.nw + SP_NT - 1) / SP_NT;
    const int w0 = threadIdx.x * per;
    const int w1 = w0 + per < A.nw ? w0 + per : A.nw;
    int cnt = 0;
    for (int m = w0; m < w1; ++m) cnt += __popcll(ld_sc(mask + m));
    total = (int)block_sum<float, SP_NT>((float)cnt, redF);
  }
  nrows = total;
  if (active) {
    lo = (int)(((int64_t)total * r) / A.R);
    hi = (int)(((int64_t)total * (r + 1)) / A.R);
  }
  select_bits(mask, A.nw, lo, hi, rowidx, redI);
  const int cnt = hi - lo;
  for (int k = threadIdx.x; k < cnt; k += SP_NT) rowval[k] = ld_sc(vec + rowidx[k]);
  __syncthreads();

  float dot = 0.f;
  if (active) {
    const int col0 = c * SP_CB;
    const int col = col0 + 4 * threadIdx.x;
    const int n = A.n;
    if (col < n) {
      const int nvalid = n - col < 4 ? n - col : 4;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const float* Qc = A.Q + col;
      int k = 0;
      if (nvalid == 4) {
        for (; k + 15 < cnt; k += 16) {
          f32x4 v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = *(const f32x4*)(Qc + (int64_t)rowidx[k + u] * n);
#pragma unroll
          for (int u = 0; u < 16; ++u) acc += rowval[k + u] * v[u];
        }
        for (; k + 3 < cnt; k += 4) {
          f32x4 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = *(const f32x4*)(Qc + (int64_t)rowidx[k + u] * n);
#pragma unroll
          for (int u = 0; u < 4; ++u) acc += rowval[k + u] * v[u];
        }
        for (; k < cnt; ++k) acc += rowval[k] * *(const f32x4*)(Qc + (int64_t)rowidx[k] * n);
      } else {
        for (; k < cnt; ++k) {
          const float* row = Qc + (int64_t)rowidx[k] * n;
          const float wv = rowval[k];
          for (int e = 0; e < nvalid; ++e) acc[e] += wv * row[e];
        }
      }
      float* dst = A.part + (int64_t)r * n + col;
      for (int e = 0; e < nvalid; ++e) {
        st_sc(dst + e, acc[e]);
        dot += acc[e] * ld_sc(vec + col + e);
      }
    }
  }
  return sp_block_sum(dot, redF);
}

// Sum over row groups of the phase-1 partials at entry i, split over the waves: wave v adds
// groups r = v, v + 4, ...; the caller combines the four wave sums.
__device__ __forceinline__ float partial_sum(const SpArgs& A, int i, int wave) {
  constexpr int NW = SP_NT / kWave;
  float s = 0.f;
  int r = wave;
  // eight independent loads in flight per round
  for (; r + 7 * NW < A.R; r += 8 * NW) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ld_sc(A.part + (int64_t)(r + u * NW) * A.n + i);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; r < A.R; r += NW) s += ld_sc(A.part + (int64_t)r * A.n + i);
  return s;
}

// Owner update of one 64-entry chunk by wave 0 after the wave sums are in LDS, publishing the
// next mask words, masked gradient, thresholds and statistics (accumulated in stats[0..3]).
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
  float s_num = wave_sum(valid ? pi * pi : 0.f);
  float s_res = wave_sum(valid ? m * m : 0.f);
  float s_cnt = wave_sum(pas ? 1.f : 0.f);
  float s_bad = wave_sum(bad ? 1.f : 0.f);
  if ((threadIdx.x & 63) == 0) {
    stats[0] += s_num;
    stats[1] += s_res;
    stats[2] += s_cnt;
    stats[3] += s_bad;
  }
}

__global__ __launch_bounds__(SP_NT) void solve_persistent_kernel(SpArgs A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int* rowidx = (int*)smem;
  float* rowval = (float*)(rowidx + A.rows_max);
  int* cidx = (int*)(rowval + A.rows_max);
  float* cval = (float*)(cidx + A.cmax);
  float* wred = cval + A.cmax;                 // [4][64] wave partials
  float* cred = wred + 4 * 64;                 // [4][64]
  float* stats = cred + 4 * 64;                // [8]
  float* redF = stats + 8;                     // [8]
  int* redI = (int*)(redF + 8);                // [8]

  const int n = A.n, G = A.G;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nchunks = A.nw;
  unsigned epoch = 0;

  // ---- start point: y = max(Y0, 0) or 0, gradient = q (refreshed below for a warm start)
  if (threadIdx.x < 8) stats[threadIdx.x] = 0.f;
  __syncthreads();
  for (int ch = blockIdx.x; ch < nchunks; ch += G) {
    if (wave == 0) {
      const int i = ch * SP_CHUNK + lane;
      const bool valid = i < n;
      float yi = 0.f, gi = 0.f;
      if (valid) {
        gi = A.q[i];
        if (A.Y0) {
          yi = A.Y0[i];
          yi = yi > 0.f ? yi : 0.f;
        }
      }
      publish_entry(A, 0, i, valid, yi, gi, ch, stats);
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) st_sc(A.scal + blockIdx.x * 8 + 1 + threadIdx.x, stats[threadIdx.x]);
  grid_barrier(A.bar, G, epoch);
  int cur = 0;

  int it = 0;
  int64_t rows = 0;  // rows of Q read by the products
  bool fresh = (A.Y0 == nullptr);
  bool need_refresh = (A.Y0 != nullptr);
  int status = NNLS_MAXITER_DEV;
  double r_now = 0.0;
  float qn2;
  {
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += SP_NT) acc += A.q[i] * A.q[i];
    qn2 = sp_block_sum(acc, redF);
  }
  const double qscale = qn2 > 0.f ? sqrt((double)qn2) : 1.0;

  for (;;) {
    if (need_refresh) {
      // gradient = Q y + q over the rows with y > 0
      int nr;
      rows_product(A, A.ymask[cur], A.y[cur], rowidx, rowval, redI, redF, nr);
      rows += nr;
      grid_barrier(A.bar, G, epoch);
      if (threadIdx.x < 8) stats[threadIdx.x] = 0.f;
      __syncthreads();
      for (int ch = blockIdx.x; ch < nchunks; ch += G) {
        const int i = ch * SP_CHUNK + lane;
        const bool valid = i < n;
        wred[wave * 64 + lane] = valid ? partial_sum(A, i, wave) : 0.f;
        __syncthreads();
        if (wave == 0) {
          const float w = wred[lane] + wred[64 + lane] + wred[128 + lane] + wred[192 + lane];
          const float yi = valid ? ld_sc(A.y[cur] + i) : 0.f;
          const float gi = valid ? A.q[i] + w : 0.f;
          publish_entry(A, cur ^ 1, i, valid, yi, gi, ch, stats);
        }
        __syncthreads();
      }
      if (threadIdx.x < 4) st_sc(A.scal + blockIdx.x * 8 + 1 + threadIdx.x, stats[threadIdx.x]);
      grid_barrier(A.bar, G, epoch);
      cur ^= 1;
      need_refresh = false;
      fresh = true;
    }

    // ---- statistics of the current iterate (same order in every workgroup)
    float num = 0.f, res = 0.f, npass = 0.f, bad = 0.f;
    {
      float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
      for (int w = threadIdx.x; w < G; w += SP_NT) {
        v0 += ld_sc(A.scal + w * 8 + 1);
        v1 += ld_sc(A.scal + w * 8 + 2);
        v2 += ld_sc(A.scal + w * 8 + 3);
        v3 += ld_sc(A.scal + w * 8 + 4);
      }
      num = sp_block_sum(v0, redF);
      res = sp_block_sum(v1, redF);
      npass = sp_block_sum(v2, redF);
      bad = sp_block_sum(v3, redF);
    }
    if (bad > 0.f) {
      status = NNLS_NONFINITE_DEV;
      break;
    }
    r_now = sqrt((double)res) / qscale;
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

    // ---- phase 1: w = Q gbar over passive rows, den shares
    int nr;
    const float den_part =
        rows_product(A, A.pmask[cur], A.p[cur], rowidx, rowval, redI, redF, nr);
    rows += nr;
    if (threadIdx.x == 0) st_sc(A.scal + blockIdx.x * 8 + 0, den_part);
    grid_barrier(A.bar, G, epoch);

    // ---- phase 2
    float den;
    {
      float v = 0.f;
      for (int w = threadIdx.x; w < G; w += SP_NT) v += ld_sc(A.scal + w * 8 + 0);
      den = sp_block_sum(v, redF);
    }
    if (!(den > 0.f) || !__builtin_isfinite(den)) {
      status = NNLS_BREAKDOWN_DEV;
      break;
    }
    const float alpha = num / den;

    // clipped set: entries with threshold y_i / gbar_i < alpha, in index order, with
    // delta_i = alpha * gbar_i - y_i.  Each thread holds the thresholds of a contiguous range
    // of SP_TPT entries in registers (all loads in flight at once).
    int ccount;
    {
      const int base = threadIdx.x * SP_TPT;
      float tv[SP_TPT];
#pragma unroll
      for (int u = 0; u < SP_TPT; ++u)
        tv[u] = (base + u < n) ? ld_sc(A.t[cur] + base + u) : __builtin_inff();
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < SP_TPT; ++u) cnt += (tv[u] < alpha);
      int pos = block_exclusive_scan<SP_NT>(cnt, redI, ccount);
#pragma unroll
      for (int u = 0; u < SP_TPT; ++u) {
        if (tv[u] < alpha) {
          cidx[pos] = base + u;
          ++pos;
        }
      }
      __syncthreads();
      rows += ccount;
      for (int m = threadIdx.x; m < ccount; m += SP_NT) {
        const int j = cidx[m];
        cval[m] = alpha * ld_sc(A.p[cur] + j) - ld_sc(A.y[cur] + j);
      }
      __syncthreads();
    }

    if (threadIdx.x < 8) stats[threadIdx.x] = 0.f;
    __syncthreads();
    for (int ch = blockIdx.x; ch < nchunks; ch += G) {
      const int i = ch * SP_CHUNK + lane;
      const bool valid = i < n;
      float wsum = 0.f, csum = 0.f;
      if (valid) {
        wsum = partial_sum(A, i, wave);
        int m = wave;
        constexpr int NW = SP_NT / kWave;
        for (; m + 3 * NW < ccount; m += 4 * NW) {
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = A.Q[(int64_t)cidx[m + u * NW] * n + i];
#pragma unroll
          for (int u = 0; u < 4; ++u) csum += cval[m + u * NW] * v[u];
        }
        for (; m < ccount; m += NW) csum += cval[m] * A.Q[(int64_t)cidx[m] * n + i];
      }
      wred[wave * 64 + lane] = wsum;
      cred[wave * 64 + lane] = csum;
      __syncthreads();
      if (wave == 0) {
        const float w = wred[lane] + wred[64 + lane] + wred[128 + lane] + wred[192 + lane];
        const float corr = cred[lane] + cred[64 + lane] + cred[128 + lane] + cred[192 + lane];
        float yi = 0.f, gi = 0.f;
        if (valid) {
          const float y0 = ld_sc(A.y[cur] + i), g0 = ld_sc(A.g[cur] + i);
          const float p0 = ld_sc(A.p[cur] + i);
          const float v = y0 - alpha * p0;
          yi = v > 0.f ? v : 0.f;
          gi = g0 - alpha * w + corr;
        }
        publish_entry(A, cur ^ 1, i, valid, yi, gi, ch, stats);
      }
      __syncthreads();
    }
    if (threadIdx.x < 4) st_sc(A.scal + blockIdx.x * 8 + 1 + threadIdx.x, stats[threadIdx.x]);
    grid_barrier(A.bar, G, epoch);
    cur ^= 1;
    ++it;
    fresh = false;
  }

  // ---- outputs
  for (int ch = blockIdx.x; ch < nchunks; ch += G) {
    if (wave == 0) {
      const int i = ch * SP_CHUNK + lane;
      if (i < n) {
        const float yi = ld_sc(A.y[cur] + i);
        A.X[i] = A.s ? (float)((double)yi / A.s[i]) : yi;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.iters[0] = it;
    A.kkt[0] = status == NNLS_NONFINITE_DEV ? __builtin_nan("") : r_now;
    A.status[0] = status;
    if (A.rows_read) A.rows_read[0] = rows;
  }
}

__global__ void solve_persistent_init_kernel(unsigned* bar) {
  for (int i = threadIdx.x; i < SP_BAR_WORDS; i += blockDim.x) bar[i] = 0u;
}

// ---- host side ------------------------------------------------------------------------------
struct SpPlan {
  int G, nb, R, nw, cmax, rows_max;
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
  P.cmax = (int)n;
  P.rows_max = (int)((n + P.R - 1) / P.R) + 1;
  P.lds = sizeof(int) * P.rows_max + sizeof(float) * P.rows_max + sizeof(int) * P.cmax +
          sizeof(float) * P.cmax + sizeof(float) * (4 * 64 * 2 + 16) + sizeof(int) * 8 + 64;
  return P;
}

// Largest n the persistent solver takes (the clipped list of up to n entries lives in LDS).
constexpr int64_t SP_MAX_N = SP_NT * SP_TPT;

bool solve_persistent_supported(int64_t n, int64_t k) {
  return k == 1 && n >= 1 && n <= SP_MAX_N && (n % 4) == 0;
}

size_t solve_persistent_ws_bytes(int64_t n) {
  const SpPlan P = sp_plan(n, sp_device_cus());
  size_t b = 0;
  b += 2 * (4 * (sizeof(float) * n + 256));       // y, g, p, t (two copies)
  b += 2 * (2 * (sizeof(uint64_t) * P.nw + 256)); // masks (two copies)
  b += sizeof(float) * (size_t)P.R * n + 256;     // partials
  b += sizeof(float) * 8 * P.G + 256;             // per-workgroup scalars
  b += sizeof(unsigned) * SP_BAR_WORDS + 256;     // barrier words
  return b + 1024;
}

hipError_t launch_solve_persistent(int64_t n, const float* Q, const float* q, const double* s,
                                   double tol, int max_iter, const float* Y0, float* X,
                                   int32_t* iters, double* kkt, int32_t* status,
                                   int64_t* rows_read, void* ws, hipStream_t st) {
  const SpPlan P = sp_plan(n, sp_device_cus());
  SpArgs A;
  A.n = (int)n;
  A.G = P.G;
  A.nb = P.nb;
  A.R = P.R;
  A.nw = P.nw;
  A.cmax = P.cmax;
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
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return (void*)r;
  };
  A.bar = (unsigned*)take(sizeof(unsigned) * SP_BAR_WORDS);
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
  hipLaunchKernelGGL(solve_persistent_init_kernel, dim3(1), dim3(256), 0, st, A.bar);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {&A};
  return hipLaunchCooperativeKernel((const void*)solve_persistent_kernel, dim3(P.G), dim3(SP_NT),
                                    args, P.lds, st);
}

}  // namespace nnls
