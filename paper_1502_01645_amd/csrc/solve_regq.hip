// Algorithm 2 for one right-hand side with Q held in the register file of the whole GPU.
//
// For n <= 5120 the rescaled matrix (at most 105 MB in FP32) fits in the vector registers of
// 256 compute units (512 KB each).  Workgroup b (one per CU, NT threads) keeps the rows
// I_b = [b RPC, (b + 1) RPC) of Q: thread t holds Q[i, j] for its columns j = t + NT s (s < CS)
// and every i in I_b, loaded once at the start.  Every workgroup also keeps the whole iterate y,
// distributed over its threads the same way, and applies the projection to all entries itself,
// so y is never exchanged.  One update e:
//   A  read the masked gradient gbar(e) at the own columns and the statistics of iterate e
//      (published by the row owners); stop test;
//   B  w_I = Q[I, :] gbar from registers; publish the partial den_b = gbar_I^T w_I;
//   C  read all partials, den = their sum (fixed order), alpha = ||gbar||^2 / den;
//      y' = [y - alpha gbar]_+ on the own columns, d = y' - y;
//   D  g'_I = g_I + Q[I, :] d (the incremental gradient of Algorithm 2); publish gbar(e + 1)
//      and the statistics of the owned rows.
// Exchange without grid barriers.  Each denominator partial is one 64-bit word with the update
// number in its high half and the FP32 value in its low half, so reading the partials is also
// the wait for them.  The gbar entries and statistics are plain coherent stores followed, once
// the wave's stores are complete, by a flag word with the update number; readers poll the G
// flags, then read the data once.  The dependencies make this safe: a workgroup overwrites its
// gbar entries (D of e) only after it has read every partial of C(e), which each workgroup
// publishes after it has finished A(e); its partial (B of e + 1) only after A(e + 1), i.e. after
// every workgroup has finished C(e).  The exact-gradient refresh before a stop is accepted is rare and uses a grid
// barrier.  Q is read from memory once per solve; an update moves the n-vector gbar and a few
// words per workgroup.  Sums over the columns of a row are per-thread FMAs, then 16-lane DPP
// row sums.
#include "common.hpp"
#include "grid_sync.hpp"
#include "kernels.hpp"

namespace nnls {


struct RqArgs {
  int n, G;
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
  float* gf;     // [CS NT] masked gradient of the current iterate, written by the row owners
                 // (entries past n stay zero)
  float* sf;     // [8 G] statistics partials
  uint64_t* fl;  // [G] publish flags: update number of the last gbar / statistics written
  uint64_t* dw;  // [G] line-search denominator partials, tagged with the update number, in
                 // RQ_DREP copies RQ_DREP_WORDS apart
  unsigned* bar;   // grid barrier words, with the abort word (grid_sync.hpp)
  int spin_limit;  // polls before a workgroup gives up waiting: a guard that never fires in a
                   // normal launch; a workgroup that gives up sets the abort word, which ends
                   // every other workgroup's waits too
};

// The denominator partials are polled by every workgroup at once; each is written to RQ_DREP
// copies far apart in memory and workgroup b polls copy b % RQ_DREP, which spreads the polling
// over several memory channels.
constexpr int RQ_DREP = 8;
constexpr int64_t RQ_DREP_WORDS = 33280;  // 260 KiB between copies

typedef __attribute__((address_space(1))) void rq_gvoid;
typedef __attribute__((address_space(3))) void rq_lvoid;
constexpr int RQ_SC1 = 16;  // cache-policy bit of an agent-coherent (sc1) load

template <int CTRL>
__device__ __forceinline__ float dpp_shr(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Inclusive sum over each 16-lane row (row_shr 1, 2, 4, 8 with zero fill): lane 15 of the row
// holds the row total.
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp_shr<0x111>(v);
  v += dpp_shr<0x112>(v);
  v += dpp_shr<0x114>(v);
  v += dpp_shr<0x118>(v);
  return v;
}

// out[r] = sum over the workgroup of acc[r], r < RPC: 16-lane row sums, then the NT / 16
// row-group partials of each r summed by 16 lanes (NT / 256 each) and a last row sum.
template <int RPC, int NT>
__device__ __forceinline__ void rows_reduce(const float (&acc)[RPC], float* red, float* out) {
  constexpr int ROWG = NT / 16;
  const int t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < RPC; ++r) {
    const float v = row16_sum(acc[r]);
    if ((t & 15) == 15) red[r * ROWG + (t >> 4)] = v;
  }
  __syncthreads();
  // 16 lanes per r; RPC * 16 may exceed NT, so the threads take the r in passes (every pass
  // and bound is a multiple of 16, so only whole 16-lane rows are active)
#pragma unroll
  for (int base = 0; base < RPC * 16; base += NT) {
    const int tt = base + t;
    if (tt < RPC * 16) {
      const int r = tt >> 4, c = tt & 15;
      float v = 0.f;
#pragma unroll
      for (int u = 0; u < ROWG / 16; ++u) v += red[r * ROWG + 16 * u + c];
      v = row16_sum(v);
      if (c == 15) out[r] = v;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ uint64_t tag(unsigned ep, float v) {
  return ((uint64_t)ep << 32) | (uint64_t)__builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ bool tag_ok(uint64_t w, unsigned ep) {
  return (unsigned)(w >> 32) == ep;
}
__device__ __forceinline__ float tag_val(uint64_t w) {
  return __builtin_bit_cast(float, (uint32_t)(w & 0xffffffffull));
}

// prod[r] = sum over the workgroup's columns of Q[i0 + r, j] v_j (v in LDS, [CS][NT])
template <int RPC, int CS, int NT>
__device__ __forceinline__ void reg_product(const float (&qr)[RPC][CS], const float* v,
                                            float* red, float* prod) {
  const int t = threadIdx.x;
  float acc[RPC];
#pragma unroll
  for (int r = 0; r < RPC; ++r) acc[r] = 0.f;
#pragma unroll
  for (int s = 0; s < CS; ++s) {
    const float x = v[s * NT + t];
#pragma unroll
    for (int r = 0; r < RPC; ++r) acc[r] += qr[r][s] * x;
  }
  rows_reduce<RPC, NT>(acc, red, prod);
}

// Workgroup shapes: RPC rows of Q per workgroup, CS columns per thread, NT threads.  With 512
// threads (two waves per SIMD) a wave has 256 registers; with 256 threads (one wave per SIMD) it
// has 512, the upper half accumulation registers that hold part of Q.  y and the vector of the
// current product (gbar, then d) live in LDS, [CS][NT].
template <int RPC, int CS, int NT>
__global__ __launch_bounds__(NT, 1) void solve_regq_kernel(RqArgs A) {
  constexpr int ROWG = NT / 16;
  __shared__ float red[RPC * ROWG];
  __shared__ float prod[RPC];
  __shared__ float redF[NT / 64];
  __shared__ float ys[CS * NT];
  __shared__ float vs[CS * NT];
  __shared__ float stl[5 * NT];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int n = A.n, G = A.G;
  const int i0 = blockIdx.x * RPC;
  const int rcnt = n - i0 <= 0 ? 0 : (n - i0 < RPC ? n - i0 : RPC);
  const bool own = t < rcnt;  // thread t < RPC owns row i0 + t

  // ---- registers: the owned rows of Q at the own columns j = t + NT s
  float qr[RPC][CS];
#pragma unroll
  for (int s = 0; s < CS; ++s) {
    const int j = t + NT * s;
#pragma unroll
    for (int r = 0; r < RPC; ++r)
      qr[r][s] = (r < rcnt && j < n) ? A.Q[(int64_t)(i0 + r) * n + j] : 0.f;
  }
#pragma unroll
  for (int s = 0; s < CS; ++s) {
    const int j = t + NT * s;
    float v = 0.f;
    if (j < n && A.Y0) v = A.Y0[j] > 0.f ? A.Y0[j] : 0.f;
    ys[s * NT + t] = v;
  }
  float g_own = own ? A.q[i0 + t] : 0.f;  // exact for the cold start
  float y_own = 0.f;
  if (own && A.Y0) y_own = A.Y0[i0 + t] > 0.f ? A.Y0[i0 + t] : 0.f;

  float qn2;
  {
    float acc = 0.f;
    for (int i = t; i < n; i += NT) acc += A.q[i] * A.q[i];
    qn2 = block_sum<float, NT>(acc, redF);
  }
  const double qscale = qn2 > 0.f ? sqrt((double)qn2) : 1.0;

  // owners publish the masked gradient of their rows and the statistics of the iterate (sum
  // gbar^2, sum min(y, g)^2, passive count, non-finite count, count y > 0), then the flag ep
  auto publish = [&](unsigned ep) {
    if (wave == 0) {
      const bool pas = own && ((y_own > 0.f) || (g_own < 0.f));
      const float p = pas ? g_own : 0.f;
      if (own) st_sc(A.gf + i0 + t, p);
      const float m = y_own < g_own ? y_own : g_own;
      const bool bad = own && (!__builtin_isfinite(y_own) || !__builtin_isfinite(g_own));
      const float s0 = wave_sum(p * p);
      const float s1 = wave_sum(own ? m * m : 0.f);
      const float s2 = wave_sum(pas ? 1.f : 0.f);
      const float s3 = wave_sum(bad ? 1.f : 0.f);
      const float s4 = wave_sum((own && y_own > 0.f) ? 1.f : 0.f);
      if (lane == 0) {
        float* dst = A.sf + blockIdx.x * 8;
        st_sc(dst + 0, s0);
        st_sc(dst + 1, s1);
        st_sc(dst + 2, s2);
        st_sc(dst + 3, s3);
        st_sc(dst + 4, s4);
      }
      __builtin_amdgcn_s_waitcnt(0);  // the wave's stores are complete before the flag
      if (lane == 0) st_sc(A.fl + blockIdx.x, (uint64_t)ep << 32);
    }
  };

  unsigned epoch = 0;      // grid barriers passed
  unsigned ep = 1;         // tag of the gbar / statistics words to read next
  unsigned ed = 1;         // tag of the denominator words to publish / read next
  bool timed_out = false;
  publish(ep);

  int it = 0;
  int64_t rows = 0;  // rows of Q an implementation streaming Q would read (|P| + |C| per update)
  int clipped = 0;   // this thread's share of the |C| terms, summed over the block at the end
  const uint64_t* dwr = A.dw + (blockIdx.x % RQ_DREP) * RQ_DREP_WORDS;
  bool fresh = (A.Y0 == nullptr);
  bool need_refresh = (A.Y0 != nullptr);
  int status = NNLS_MAXITER_DEV;
  double r_now = 0.0;
  float st5[5];

  // A: wait for every flag to carry ep, then gbar at the own columns into vs and the five
  // statistics summed over the workgroups (one 5-wide reduction)
  __shared__ float red5[5][NT / 64];
  auto read_gbar = [&]() -> bool {
    for (int poll = 0;; ++poll) {
      const bool ok = t >= G || tag_ok(ld_sc(A.fl + t), ep);
      if (__syncthreads_and(ok)) break;
      // (poll is the same in every thread, so either all threads reach the _or or none)
      if (poll >= A.spin_limit ||
          ((poll & 63) == 63 && __syncthreads_or(t == 0 && grid_aborted(A.bar)))) {
        if (t == 0) grid_abort(A.bar);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // gbar at the own columns straight into vs, and the statistics of every workgroup into
    // stl, by global-to-LDS loads with the agent-coherent cache policy (sc1, the policy of the
    // agent-scope loads): a thread's CS + 5 loads are all in flight at once and never pass
    // through registers (agent-scope atomic loads would each wait for the previous one).
    // gf is zero-padded to CS x NT entries; rows of stl past G read workgroup 0's words and are
    // ignored.
    // (the lane offsets are made opaque here so that the addresses are formed at each read as
    // uniform base + lane offset instead of being kept in registers through the whole solve)
    const int wl = wave * 64;
    int tg = t, tc = t < G ? 8 * t : 0;
    asm volatile("" : "+v"(tg), "+v"(tc));
#pragma unroll
    for (int s = 0; s < CS; ++s)
      __builtin_amdgcn_global_load_lds((rq_gvoid*)(A.gf + NT * s + tg),
                                       (rq_lvoid*)(vs + s * NT + wl), 4, 0, RQ_SC1);
#pragma unroll
    for (int u = 0; u < 5; ++u)
      __builtin_amdgcn_global_load_lds((rq_gvoid*)(A.sf + u + tc), (rq_lvoid*)(stl + u * NT + wl),
                                       4, 0, RQ_SC1);
    __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0), lgkmcnt(0)
    __syncthreads();
    float sv[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) sv[u] = wave_sum(t < G ? stl[u * NT + t] : 0.f);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < 5; ++u) red5[u][wave] = sv[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      float a = 0.f;
#pragma unroll
      for (int v = 0; v < NT / 64; ++v) a += red5[u][v];
      st5[u] = a;
    }
    __syncthreads();
    return true;
  };

  for (;;) {
    if (!read_gbar()) {
      timed_out = true;
      break;
    }
    if (need_refresh) {
      // exact gradient g_I = q_I + Q[I, :] y; everyone has finished reading gbar(ep) before
      // the owners overwrite it
      rows += (int64_t)st5[4];
      if (!grid_barrier(A.bar, G, epoch, A.spin_limit)) {
        timed_out = true;
        break;
      }
      reg_product<RPC, CS, NT>(qr, ys, red, prod);
      if (own) g_own = A.q[i0 + t] + prod[t];
      publish(++ep);
      need_refresh = false;
      fresh = true;
      continue;
    }
    const float num = st5[0], res = st5[1], npass = st5[2], bad = st5[3];
    if (bad > 0.f) {
      status = NNLS_NONFINITE_DEV;
      break;
    }
    r_now = sqrt((double)res) / qscale;
    if (A.trace != nullptr && blockIdx.x == 0 && t == 0 && it < A.trace_len) {
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

    // ---- B: w_I = Q[I, :] gbar, den partial
    reg_product<RPC, CS, NT>(qr, vs, red, prod);
    const float w_own = own ? prod[t] : 0.f;
    if (wave == 0) {
      const bool pas = own && ((y_own > 0.f) || (g_own < 0.f));
      const float v = wave_sum(pas ? g_own * prod[t] : 0.f);
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < RQ_DREP; ++r) st_sc(A.dw + r * RQ_DREP_WORDS + blockIdx.x, tag(ed, v));
      }
    }

    // ---- C: den (the same in every workgroup: fixed-order sums of the same partials)
    float den = 0.f;
    {
      bool got = false;
      for (int poll = 0;; ++poll) {
        bool ok = true;
        float v = 0.f;
        for (int c = t; c < G; c += NT) {
          const uint64_t w = ld_sc(dwr + c);
          ok = ok && tag_ok(w, ed);
          v += tag_val(w);
        }
        if (__syncthreads_and(ok)) {
          den = block_sum<float, NT>(v, redF);
          got = true;
          break;
        }
        if (poll >= A.spin_limit ||
            ((poll & 63) == 63 && __syncthreads_or(t == 0 && grid_aborted(A.bar))))
          break;
        __builtin_amdgcn_s_sleep(2);
      }
      if (!got) {
        if (t == 0) grid_abort(A.bar);
        timed_out = true;
        break;
      }
    }
    ++ed;
    if (!(den > 0.f) || !__builtin_isfinite(den)) {
      status = NNLS_BREAKDOWN_DEV;
      break;
    }
    const float alpha = num / den;

    // projection on the own columns (a thread reads and writes only its own entries of ys and
    // vs, so no barrier is needed).  With v = y - alpha gbar, d = y' - y = -alpha gbar + c where
    // c = -v on the clipped entries and 0 elsewhere; vs becomes c.
#pragma unroll
    for (int s = 0; s < CS; ++s) {
      const float yo = ys[s * NT + t];
      const float v = yo - alpha * vs[s * NT + t];
      const bool clip = v < 0.f;
      clipped += clip ? 1 : 0;
      vs[s * NT + t] = clip ? -v : 0.f;
      ys[s * NT + t] = clip ? 0.f : v;
    }

    // ---- D: g'_I = g_I + Q[I, :] d = g_I - alpha w_I + Q[I, :] c, publish gbar(e + 1); the
    // product runs over the clipped columns only
    {
      float acc[RPC];
#pragma unroll
      for (int r = 0; r < RPC; ++r) acc[r] = 0.f;
#pragma unroll
      for (int s = 0; s < CS; ++s) {
        const float c = vs[s * NT + t];
        if (c != 0.f) {
#pragma unroll
          for (int r = 0; r < RPC; ++r) acc[r] += qr[r][s] * c;
        }
      }
      rows_reduce<RPC, NT>(acc, red, prod);
    }
    if (own) {
      g_own = (g_own - alpha * w_own) + prod[t];
      const int i = i0 + t;
      y_own = ys[(i / NT) * NT + (i % NT)];
    }
    publish(++ep);
    ++it;
    fresh = false;
  }

  // ---- outputs
  rows += (int64_t)block_sum<float, NT>((float)clipped, redF);
  if (own) A.X[i0 + t] = A.s ? (float)((double)y_own / A.s[i0 + t]) : y_own;
  if (blockIdx.x == 0 && t == 0) {
    A.iters[0] = timed_out ? -1 : it;
    A.kkt[0] = (status == NNLS_NONFINITE_DEV || timed_out) ? __builtin_nan("") : r_now;
    A.status[0] = timed_out ? NNLS_BREAKDOWN_DEV : status;
    if (A.rows_read) A.rows_read[0] = rows;
  }
}

// Zeroes the barrier words, the flags and every copy of the denominator partials (tag 0 never
// matches a read), and the gradient exchange vector (its entries past n are read as padding).
__global__ void regq_init_kernel(unsigned* bar, uint64_t* fl, uint64_t* dw, int G, float* gf,
                                 int64_t ngf) {
  for (int i = threadIdx.x; i < GS_BAR_WORDS; i += blockDim.x) bar[i] = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)G * (RQ_DREP + 1);
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / G, c = i % G;
    if (r == 0) fl[c] = 0ull;
    else dw[(r - 1) * RQ_DREP_WORDS + c] = 0ull;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ngf;
       i += (int64_t)gridDim.x * blockDim.x)
    gf[i] = 0.f;
}

// ---- host side ------------------------------------------------------------------------------
namespace {

struct RqShape {
  int rpc, cs, nt;
};
constexpr RqShape kRqShapes[] = {{8, 4, 512}, {12, 6, 512}, {16, 8, 512}, {20, 20, 256}};
constexpr int RQ_GF = 5120;  // entries of the gradient exchange vector: CS x NT of every shape
static_assert(4 * 512 <= RQ_GF && 6 * 512 <= RQ_GF && 8 * 512 <= RQ_GF && 20 * 256 <= RQ_GF,
              "exchange vector too short for a shape");

int rq_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

int rq_pick(int64_t n, int G) {
  for (int i = 0; i < (int)(sizeof(kRqShapes) / sizeof(kRqShapes[0])); ++i)
    if ((int64_t)kRqShapes[i].rpc * G >= n && (int64_t)kRqShapes[i].cs * kRqShapes[i].nt >= n &&
        kRqShapes[i].nt >= G && G <= RQ_DREP_WORDS)
      return i;
  return -1;
}

template <int RPC, int CS, int NT>
hipError_t rq_launch(RqArgs& A, hipStream_t st) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, (const void*)solve_regq_kernel<RPC, CS, NT>, NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  void* args[] = {&A};
  return hipLaunchCooperativeKernel((const void*)solve_regq_kernel<RPC, CS, NT>, dim3(A.G),
                                    dim3(NT), args, 0, st);
}

}  // namespace

bool solve_regq_supported(int64_t n, int64_t k) {
  if (k != 1 || n < 1) return false;
  const int G = rq_cus();
  return G > 0 && rq_pick(n, G) >= 0;
}

size_t solve_regq_ws_bytes(int64_t n) {
  const int G = rq_cus() > 0 ? rq_cus() : 1;
  (void)n;
  return sizeof(unsigned) * GS_BAR_WORDS + 256 + sizeof(uint64_t) * (size_t)G + 256 +
         sizeof(uint64_t) * RQ_DREP * (size_t)RQ_DREP_WORDS + 256 +
         sizeof(float) * (RQ_GF + 8 * (size_t)G) + 512;
}

hipError_t launch_solve_regq(int64_t n, const float* Q, const float* q, const double* s,
                             double tol, int max_iter, const float* Y0, float* X, int32_t* iters,
                             double* kkt, int32_t* status, int64_t* rows_read, float* trace,
                             int trace_len, void* ws, hipStream_t st) {
  const int G = rq_cus();
  const int pick = G > 0 ? rq_pick(n, G) : -1;
  if (pick < 0) return hipErrorInvalidValue;
  RqArgs A;
  A.n = (int)n;
  A.G = G;
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
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return (void*)r;
  };
  A.bar = (unsigned*)take(sizeof(unsigned) * GS_BAR_WORDS);
  A.fl = (uint64_t*)take(sizeof(uint64_t) * (size_t)G);
  A.dw = (uint64_t*)take(sizeof(uint64_t) * RQ_DREP * (size_t)RQ_DREP_WORDS);
  A.gf = (float*)take(sizeof(float) * RQ_GF);
  A.sf = (float*)take(sizeof(float) * 8 * (size_t)G);
  A.spin_limit = spin_limit_setting();
  hipLaunchKernelGGL(regq_init_kernel, dim3(8), dim3(256), 0, st, A.bar, A.fl, A.dw, G, A.gf,
                     (int64_t)RQ_GF);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (pick) {
    case 0: return rq_launch<8, 4, 512>(A, st);
    case 1: return rq_launch<12, 6, 512>(A, st);
    case 2: return rq_launch<16, 8, 512>(A, st);
    default: return rq_launch<20, 20, 256>(A, st);
  }
}

}  // namespace nnls
