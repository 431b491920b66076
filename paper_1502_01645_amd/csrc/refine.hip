// FP64 check and one refinement step against the original data (A, B).
//
// In the rescaled variables y = s .* x (s_i = ||A_i||), with g = A^T (A x - B) = H x - A^T B:
//   grad_y = g ./ s, passive set, masked gradient p, relative KKT residual
//   ||min(y, grad_y)|| / ||A^T b ./ s||; direction D = p ./ s, exact step
//   alpha = ||p||^2 / (D^T H D) (= p^T Q p), candidate x' = [x - alpha D]_+; keep x' when it lowers
//   the residual without raising F(x) = 1/2 ||A x - b||^2, and report the residual and objective
//   of the x that is returned.
// Few right-hand sides (k <= 4) stream A once per pass with matrix-vector kernels:
//   R = A X - B, g = A^T R, V = A D (D^T H D = ||V||^2), R' = A x' - B, g' = A^T R'.
// For one right-hand side and n <= 6144 (FP32 A, aligned rows) a workgroup holds a few full rows
// of A in registers, forms their residuals and adds their share of A^T R before it moves on, so
// (R, g) and (R', g') each cost one read of A: three reads instead of five.
// Many right-hand sides form the FP64 Gram matrix once, on the FP64 matrix cores:
//   H = A^T A, a = A^T B;  g = H X - a,  D^T H D from H D,  g' = H X' - a,
//   F(x') - F(x) = 1/2 (x' - x)^T (g + g') for the keep decision,
// so the work over the d rows of A is one product instead of five.  The objective that is
// reported, F = 1/2 ||A x - b||^2 of the returned x, comes from the residuals R = A X - B (one
// more FP64 product, only when the caller asks for it): the Gram form
// 1/2 (x^T (H x - 2 a) + ||b||^2) loses every digit of F near a noiseless fit, where its three
// terms are each about 1/2 ||b||^2 and F is not.
#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int RF_SMALL_K = 4;

// ---- few right-hand sides --------------------------------------------------------------------
// out[r, c] = sum_i A[r, i] X[i, c] - B[r, c] for c < k (k <= RF_SMALL_K); one wave per row.
template <typename TA, typename TX>
__global__ __launch_bounds__(256) void rows_residual_kernel(int64_t d, int64_t n, int64_t k,
                                                            const TA* __restrict__ A, int64_t lda,
                                                            const TX* __restrict__ X,
                                                            const TA* __restrict__ B, int64_t ldb,
                                                            double* __restrict__ R) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= d) return;
  double acc[RF_SMALL_K];
#pragma unroll
  for (int c = 0; c < RF_SMALL_K; ++c) acc[c] = 0.0;
  const TA* row = A + r * lda;
  for (int64_t i = lane; i < n; i += 64) {
    const double a = (double)row[i];
#pragma unroll
    for (int c = 0; c < RF_SMALL_K; ++c)
      if (c < k) acc[c] += a * (double)X[i * k + c];
  }
#pragma unroll
  for (int c = 0; c < RF_SMALL_K; ++c) {
    if (c < k) {
      const double v = wave_sum(acc[c]);
      if (lane == 0) R[r * k + c] = v - (B ? (double)B[r * ldb + c] : 0.0);
    }
  }
}

// Vectorized form of the same product for FP32 A with 16-byte aligned rows (lda % 4 == 0): each
// wave takes RPW rows at once, each lane 4 consecutive columns per step, so one load of x serves
// RPW rows and RPW independent 16-byte loads of A are in flight per step.  KV is the number of
// right-hand sides the registers are sized for (k <= KV): 1 leaves room for 8 rows per wave.
constexpr int RF_RPW = 4;
constexpr int RF_RPW1 = 8;

template <typename TX>
__device__ __forceinline__ void load_x4(const TX* X, int64_t i, int64_t k, int c, double* xv) {
#pragma unroll
  for (int e = 0; e < 4; ++e) xv[e] = (double)X[(i + e) * k + c];
}

template <typename TX, int KV, int RPW>
__global__ __launch_bounds__(256) void rows_residual_vec_kernel(int64_t d, int64_t n, int64_t k,
                                                                const float* __restrict__ A,
                                                                int64_t lda,
                                                                const TX* __restrict__ X,
                                                                const float* __restrict__ B,
                                                                int64_t ldb,
                                                                double* __restrict__ R) {
  const int lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
  if (r0 >= d) return;
  double acc[RPW][KV];
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int c = 0; c < KV; ++c) acc[q][c] = 0.0;
  for (int64_t i = 4 * lane; i < n; i += 256) {
    f32x4 a[RPW];
#pragma unroll
    for (int q = 0; q < RPW; ++q)
      a[q] = (r0 + q < d) ? *(const f32x4*)(A + (r0 + q) * lda + i) : (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KV; ++c) {
      if (c < k) {
        double xv[4];
        load_x4(X, i, k, c, xv);
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[q][c] += (double)a[q][e] * xv[e];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
#pragma unroll
    for (int c = 0; c < KV; ++c) {
      if (c < k) {
        const double v = wave_sum(acc[q][c]);
        if (lane == 0 && r0 + q < d)
          R[(r0 + q) * k + c] = v - (B ? (double)B[(r0 + q) * ldb + c] : 0.0);
      }
    }
  }
}

// Vectorized A^T V for FP32 A with aligned rows: each thread owns 4 consecutive columns of a
// 1024-column block and walks the rows of its chunk 8 at a time (8 independent 16-byte loads in
// flight).  Same partial layout as cols_partial_kernel.
template <int KV>
__global__ __launch_bounds__(256) void cols_partial_vec_kernel(int64_t d, int64_t n,
                                                               const float* __restrict__ A,
                                                               int64_t lda,
                                                               const double* __restrict__ R,
                                                               const float* __restrict__ B,
                                                               int64_t ldb, int with_b,
                                                               int64_t rows_per_chunk,
                                                               double* __restrict__ partial) {
  constexpr int k = KV;
  const int64_t i = (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (i >= n) return;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < d ? r0 + rows_per_chunk : d;
  const int nvec = with_b ? 2 * k + 1 : k;
  double acc[2 * KV + 1][4];
#pragma unroll
  for (int m = 0; m < 2 * KV + 1; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[m][e] = 0.0;
  int64_t r = r0;
  for (; r + 7 < r1; r += 8) {
    f32x4 a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = *(const f32x4*)(A + (r + u) * lda + i);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int c = 0; c < k; ++c) {
        const double rv = R[(r + u) * k + c];
        const double bv = with_b ? (double)B[(r + u) * ldb + c] : 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[c][e] += (double)a[u][e] * rv;
          if (with_b) acc[k + c][e] += (double)a[u][e] * bv;
        }
      }
      if (with_b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[2 * k][e] += (double)a[u][e] * (double)a[u][e];
      }
    }
  }
  for (; r < r1; ++r) {
    const f32x4 a = *(const f32x4*)(A + r * lda + i);
#pragma unroll
    for (int c = 0; c < k; ++c) {
      const double rv = R[r * k + c];
      const double bv = with_b ? (double)B[r * ldb + c] : 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[c][e] += (double)a[e] * rv;
        if (with_b) acc[k + c][e] += (double)a[e] * bv;
      }
    }
    if (with_b) {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[2 * k][e] += (double)a[e] * (double)a[e];
    }
  }
  for (int m = 0; m < nvec; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) partial[(chunk * nvec + m) * n + i + e] = acc[m][e];
}

// One right-hand side, fused: R[r] = sum_i A[r, i] x_i - b_r for the rows of this workgroup's
// range, and partial[wg, m, i] = sum over those rows of A[r, i] v_m[r] with v_0 = R, and with WB
// v_1 = b and v_2 = A[r, i] (the squared column norm), in the layout of cols_partial_vec_kernel
// with one chunk per workgroup.  Thread t owns columns 2048 j + 4 t .. + 3 (j < NB); a step takes
// RC_RB rows: each thread's share of their dot products, a wave sum, then a sum over the eight
// waves through LDS (double-buffered, one barrier per step) gives the residuals, and the rows
// still in registers are added into the column sums.  The rows of the next PF - 1 steps are in
// flight meanwhile (a ring of PF register buffers, rotated by unrolling the step loop PF times),
// so HBM reads continue across the reductions.  x holds FP32 values (for TX = double, values
// rounded to FP32, as the candidate x' of the refinement is); the products are exact in FP64.
constexpr int RC_NT = 512;
constexpr int RC_RB = 2;
constexpr int RC_MAX_NB = 3;
constexpr int RC_MAX_WG = 256;
// steps in flight: as many as the registers hold next to the column sums
constexpr int rc_pf(int nb, bool wb) { return nb == 1 ? 4 : (wb ? (nb == 3 ? 3 : 4) : 4); }

template <int NB, bool WB, typename TX>
__global__ __launch_bounds__(RC_NT, 1) void rows_cols_fused_kernel(
    int64_t d, int64_t n, const float* __restrict__ A, int64_t lda, const TX* __restrict__ X,
    const float* __restrict__ B, int64_t ldb, int64_t rows_per_wg, double* __restrict__ R,
    double* __restrict__ partial) {
  constexpr int NV = WB ? 3 : 1;
  constexpr int PF = rc_pf(NB, WB);
  __shared__ double red[2][RC_NT / 64][RC_RB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = r0 + rows_per_wg < d ? r0 + rows_per_wg : d;
  if (r0 >= d) return;  // whole workgroup (uniform)
  bool cv[NB];
  float xv[NB][4];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int64_t c = 2048 * j + 4 * tid;
    cv[j] = c < n;
#pragma unroll
    for (int e = 0; e < 4; ++e) xv[j][e] = cv[j] ? (float)X[c + e] : 0.f;
  }
  double acc[NV][NB][4];
#pragma unroll
  for (int m = 0; m < NV; ++m)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[m][j][e] = 0.0;

  f32x4 a[PF][RC_RB][NB];
  float bq[PF][RC_RB];
  auto load_step = [&](int64_t rs, f32x4 (&av)[RC_RB][NB], float (&bv)[RC_RB]) {
#pragma unroll
    for (int q = 0; q < RC_RB; ++q) {
      const bool rv = rs + q < r1;
#pragma unroll
      for (int j = 0; j < NB; ++j)
        av[q][j] = (rv && cv[j]) ? *(const f32x4*)(A + (rs + q) * lda + 2048 * j + 4 * tid)
                                 : (f32x4){0.f, 0.f, 0.f, 0.f};
      bv[q] = rv ? B[(rs + q) * ldb] : 0.f;
    }
  };
  auto process = [&](int64_t rs, const f32x4 (&av)[RC_RB][NB], const float (&bv)[RC_RB],
                     int par) {
    double dot[RC_RB];
#pragma unroll
    for (int q = 0; q < RC_RB; ++q) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) t += (double)av[q][j][e] * (double)xv[j][e];
      dot[q] = wave_sum(t);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < RC_RB; ++q) red[par][wave][q] = dot[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RC_RB; ++q) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < RC_NT / 64; ++w) t += red[par][w][q];
      // rows past the range have zero A and b, so their residual is 0 and adds nothing
      const double rq = t - (double)bv[q];
      if (tid == q && rs + q < r1) R[rs + q] = rq;
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double x = (double)av[q][j][e];
          acc[0][j][e] += x * rq;
          if (WB) {
            acc[1 % NV][j][e] += x * (double)bv[q];
            acc[2 % NV][j][e] += x * x;
          }
        }
    }
  };

#pragma unroll
  for (int p = 0; p + 1 < PF; ++p)
    if (r0 + p * RC_RB < r1) load_step(r0 + p * RC_RB, a[p], bq[p]);
  // step u of a round uses buffer u; the buffer it refills, (u + PF - 1) % PF, was used by the
  // step before; the LDS parity alternates with the step (PF * round + u), so PF even keeps it
  // a compile-time value and PF odd flips it once per round
  int round_par = 0;
  for (int64_t rs = r0; rs < r1; rs += PF * RC_RB) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int64_t rc = rs + u * RC_RB;
      if (rc >= r1) break;
      const int64_t rn = rc + (PF - 1) * RC_RB;
      if (rn < r1) load_step(rn, a[(u + PF - 1) % PF], bq[(u + PF - 1) % PF]);
      process(rc, a[u], bq[u], (round_par + u) & 1);
    }
    round_par ^= PF & 1;
  }
#pragma unroll
  for (int m = 0; m < NV; ++m)
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (cv[j]) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          partial[((int64_t)blockIdx.x * NV + m) * n + 2048 * j + 4 * tid + e] = acc[m][j][e];
      }
}

// partial[chunk, m, i] = sum over rows of the chunk of A[r, i] * V_m[r] where the m-th vector is
// column m of R (m < k), column m - k of B (k <= m < 2k), and A[r, i] itself (m = 2k, giving the
// squared column norm).  nvec = 2k + 1 when with_b, else k.
template <typename TA>
__global__ __launch_bounds__(256) void cols_partial_kernel(int64_t d, int64_t n, int64_t k,
                                                           const TA* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ R,
                                                           const TA* __restrict__ B, int64_t ldb,
                                                           int with_b, int64_t rows_per_chunk,
                                                           double* __restrict__ partial) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (i >= n) return;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < d ? r0 + rows_per_chunk : d;
  const int nvec = with_b ? (int)(2 * k + 1) : (int)k;
  double acc[2 * RF_SMALL_K + 1];
#pragma unroll
  for (int m = 0; m < 2 * RF_SMALL_K + 1; ++m) acc[m] = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double a = (double)A[r * lda + i];
#pragma unroll
    for (int c = 0; c < RF_SMALL_K; ++c) {
      if (c < k) {
        acc[c] += a * R[r * k + c];
        if (with_b) acc[k + c] += a * (double)B[r * ldb + c];
      }
    }
    if (with_b) acc[2 * k] += a * a;
  }
  for (int m = 0; m < nvec; ++m) partial[(chunk * nvec + m) * n + i] = acc[m];
}

// Block: 16 columns x all nvec vectors; thread (column tid % 16, group tid / 16) sums the chunks
// g, g + 16, ... with four accumulators, then the 16 group sums of a column are added in fixed
// order.  (A wave reads 16 consecutive doubles of 4 chunks at a time; 16 columns per block give
// enough blocks to spread the partial sums over the GPU.)
constexpr int CF_C = 16;
constexpr int CF_G = 256 / CF_C;
__global__ __launch_bounds__(256) void cols_finalize_kernel(int64_t n, int64_t k, int with_b,
                                                            int64_t nchunks,
                                                            const double* __restrict__ partial,
                                                            double* __restrict__ G,
                                                            double* __restrict__ Atb,
                                                            double* __restrict__ s) {
  __shared__ double red[CF_G][CF_C];
  const int cl = threadIdx.x % CF_C, grp = threadIdx.x / CF_C;
  const int64_t i = (int64_t)blockIdx.x * CF_C + cl;
  const int nvec = with_b ? (int)(2 * k + 1) : (int)k;
  for (int m = 0; m < nvec; ++m) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
      int64_t c = grp;
      for (; c + 3 * CF_G < nchunks; c += 4 * CF_G) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += partial[((c + CF_G * u) * nvec + m) * n + i];
      }
      for (; c < nchunks; c += CF_G) a[0] += partial[(c * nvec + m) * n + i];
    }
    red[grp][cl] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    if (grp == 0 && i < n) {
      double acc = 0.0;
#pragma unroll
      for (int g = 0; g < CF_G; ++g) acc += red[g][cl];
      if (m < k) G[i * k + m] = acc;
      else if (m < 2 * k) Atb[i * k + (m - k)] = acc;
      else s[i] = acc > 0.0 ? sqrt(acc) : 1.0;
    }
    __syncthreads();
  }
}

// ---- many right-hand sides: FP64 Gram path ---------------------------------------------------
// C[i, j] = sum_r A[r, i] M[r, j] for i < N, r < K, with M = [M1 | M2] (columns j < n1 from M1,
// the next n2 from M2; all row-major with r as the row), written to C1 (j < n1) and C2 (the rest)
// in FP64 on the matrix cores (v_mfma_f64_16x16x4f64): 64 x 64 output tiles, four waves of
// 32 x 32, K staged through LDS 32 rows at a time (zero-filled past the edges) with the next
// chunk loaded into registers while the current one is multiplied.
// Split over K (part != nullptr): workgroup z of gridDim.z takes rows [z kps, (z + 1) kps) of the
// sum and writes its partial tile to part[z][i][j] (j over all n1 + n2 columns);
// gemm_tn_reduce_kernel adds the partials in order of z.
// Four workgroups per CU (126 registers, 4 x 36 KB of LDS): 3-4 % faster than three.
constexpr int TN_T = 64, TN_BK = 32, TN_LD = TN_T + 2;

template <typename TA, typename TM>
__global__ __launch_bounds__(256, 4) void gemm_tn_f64_kernel(
    int64_t K, int64_t N, int64_t n1, int64_t n2, const TA* __restrict__ A, int64_t lda,
    const TM* __restrict__ M1, int64_t ld1, const TM* __restrict__ M2, int64_t ld2,
    double* __restrict__ C1, int64_t ldc1, double* __restrict__ C2, int64_t ldc2, int64_t kps,
    double* __restrict__ part) {
  __shared__ double sa[TN_BK][TN_LD];
  __shared__ double sm[TN_BK][TN_LD];
  const int64_t i0 = (int64_t)blockIdx.y * TN_T, j0 = (int64_t)blockIdx.x * TN_T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // staging: this thread's column c = tid % 64, rows (tid / 64) + 4 u of each chunk
  const int c = tid & 63, r0 = tid >> 6;
  const int64_t ia = i0 + c, jm = j0 + c;
  const bool a_ok = ia < N;
  const TM* mp = nullptr;
  int64_t mld = 0;
  if (jm < n1) {
    mp = M1 + jm;
    mld = ld1;
  } else if (jm < n1 + n2) {
    mp = M2 + (jm - n1);
    mld = ld2;
  }
  TA ra[TN_BK / 4];
  TM rm[TN_BK / 4];
  // rows [kb, ke) of the sum: all of them, or this split's share
  const int64_t kb = part != nullptr ? (int64_t)blockIdx.z * kps : 0;
  const int64_t ke = part != nullptr ? (kb + kps < K ? kb + kps : K) : K;
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < TN_BK / 4; ++u) {
      const int64_t gr = k0 + r0 + 4 * u;
      ra[u] = (a_ok && gr < ke) ? A[gr * lda + ia] : (TA)0;
      rm[u] = (mp != nullptr && gr < ke) ? mp[gr * mld] : (TM)0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < TN_BK / 4; ++u) {
      sa[r0 + 4 * u][c] = (double)ra[u];
      sm[r0 + 4 * u][c] = (double)rm[u];
    }
  };

  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const int col = lane & 15, kq = lane >> 4;
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += TN_BK) {
    store();
    __syncthreads();
    if (k0 + TN_BK < ke) load(k0 + TN_BK);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < TN_BK; kk += 4) {
      const int kr = kk + kq;
      const double a0 = sa[kr][wi + col], a1 = sa[kr][wi + 16 + col];
      const double b0 = sm[kr][wj + col], b1 = sm[kr][wj + 16 + col];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane l holds column l % 16 and rows l / 16 + 4 e of each 16 x 16 block (the FP64 layout;
  // the FP32 16 x 16 instructions place rows 4 (l / 16) + e instead)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = i0 + wi + a * 16 + kq + 4 * e;
        const int64_t j = j0 + wj + b * 16 + col;
        if (i >= N) continue;
        if (part != nullptr) {
          if (j < n1 + n2) part[((int64_t)blockIdx.z * N + i) * (n1 + n2) + j] = acc[a][b][e];
        } else if (j < n1) {
          C1[i * ldc1 + j] = acc[a][b][e];
        } else if (j < n1 + n2) {
          C2[i * ldc2 + (j - n1)] = acc[a][b][e];
        }
      }
}

// C1 / C2 from the split partials of gemm_tn_f64_kernel: element e of the N x (n1 + n2) result
// is the sum over z < S of its partials, in order of z.
__global__ __launch_bounds__(256) void gemm_tn_reduce_kernel(
    int S, int64_t N, int64_t n1, int64_t n2, const double* __restrict__ part,
    double* __restrict__ C1, int64_t ldc1, double* __restrict__ C2, int64_t ldc2) {
  const int64_t w = n1 + n2, tot = N * w;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < tot) {
    double v = 0.0;
    for (int z = 0; z < S; ++z) v += part[(int64_t)z * tot + e];
    const int64_t i = e / w, j = e % w;
    if (j < n1) C1[i * ldc1 + j] = v;
    else C2[i * ldc2 + (j - n1)] = v;
  }
}

// s_i = sqrt(H_ii), 1 where H_ii = 0.
__global__ void diag_scale_kernel(int64_t n, const double* __restrict__ H, double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const double h = H[i * n + i];
    s[i] = h > 0.0 ? sqrt(h) : 1.0;
  }
}

// Per-column stages of the Gram path: 16 columns per block, thread t on column t % 16 and rows
// t / 16, t / 16 + 16, ... (a wave reads 16 consecutive columns of 4 rows; 16 columns per block
// give k / 16 blocks, enough to spread k = 4096 over the GPU).
constexpr int GS_C = 16;
constexpr int GS_G = 256 / GS_C;  // row groups

// Sum over the GS_G row groups of a column, pairwise in a fixed order; every thread gets it.
__device__ __forceinline__ double gs_reduce(double v, double (*red)[GS_C], int rg, int cl) {
  red[rg][cl] = v;
  __syncthreads();
  double t[GS_G / 2];
#pragma unroll
  for (int g = 0; g < GS_G / 2; ++g) t[g] = red[2 * g][cl] + red[2 * g + 1][cl];
#pragma unroll
  for (int w = GS_G / 4; w >= 1; w >>= 1)
#pragma unroll
    for (int g = 0; g < w; ++g) t[g] = t[2 * g] + t[2 * g + 1];
  __syncthreads();
  return t[0];
}

// Stage 1: residual at x, direction D = p ./ s, ||p||^2.
template <typename TX>
__global__ __launch_bounds__(256) void gref_stage1_kernel(int64_t n, int64_t k,
                                                          const TX* __restrict__ X,
                                                          const double* __restrict__ GX,
                                                          const double* __restrict__ Atb,
                                                          const double* __restrict__ s,
                                                          double* __restrict__ D,
                                                          double* __restrict__ colstat) {
  __shared__ double red[GS_G][GS_C];
  const int cl = threadIdx.x % GS_C, rg = threadIdx.x / GS_C;
  const int64_t c = (int64_t)blockIdx.x * GS_C + cl;
  const bool in = c < k;
  double kk = 0.0, aa = 0.0, num = 0.0;
  if (in) {
    for (int64_t i = rg; i < n; i += GS_G) {
      const int64_t o = i * k + c;
      const double x = (double)X[o], a = Atb[o], hx = GX[o], si = s[i];
      const double y = si * x, gy = (hx - a) / si;
      const double p = (y > 0.0 || gy < 0.0) ? gy : 0.0;
      num += p * p;
      D[o] = p / si;
      const double m = y < gy ? y : gy;
      kk += m * m;
      const double ai = a / si;
      aa += ai * ai;
    }
  }
  kk = gs_reduce(kk, red, rg, cl);
  aa = gs_reduce(aa, red, rg, cl);
  num = gs_reduce(num, red, rg, cl);
  if (in && rg == 0) {
    colstat[c * 8 + 0] = aa > 0.0 ? sqrt(kk) / sqrt(aa) : sqrt(kk);
    colstat[c * 8 + 2] = num;
    colstat[c * 8 + 3] = aa;
  }
}

// Stage 2 (after HD = H D): alpha = ||p||^2 / D^T H D and the candidate x' (rounded to TX).
template <typename TX>
__global__ __launch_bounds__(256) void gref_stage2_kernel(int64_t n, int64_t k,
                                                          const TX* __restrict__ X,
                                                          const double* __restrict__ D,
                                                          const double* __restrict__ HD,
                                                          double* __restrict__ Xn,
                                                          const double* __restrict__ colstat) {
  __shared__ double red[GS_G][GS_C];
  const int cl = threadIdx.x % GS_C, rg = threadIdx.x / GS_C;
  const int64_t c = (int64_t)blockIdx.x * GS_C + cl;
  const bool in = c < k;
  double den = 0.0;
  if (in)
    for (int64_t i = rg; i < n; i += GS_G) den += D[i * k + c] * HD[i * k + c];
  den = gs_reduce(den, red, rg, cl);
  if (!in) return;
  const double num = colstat[c * 8 + 2];
  const double alpha = (den > 0.0 && __builtin_isfinite(den)) ? num / den : 0.0;
  for (int64_t i = rg; i < n; i += GS_G) {
    const int64_t o = i * k + c;
    const double v = (double)X[o] - alpha * D[o];
    Xn[o] = (double)(TX)(v > 0.0 ? v : 0.0);
  }
}

// Stage 3 (after HXn = H x'): residual at x', objective change, accept or reject, results.
template <typename TX>
__global__ __launch_bounds__(256) void gref_stage3_kernel(int64_t n, int64_t k,
                                                          TX* __restrict__ X,
                                                          const double* __restrict__ Xn,
                                                          const double* __restrict__ HXn,
                                                          const double* __restrict__ GX,
                                                          const double* __restrict__ Atb,
                                                          const double* __restrict__ s,
                                                          const double* __restrict__ colstat,
                                                          double* __restrict__ kkt64) {
  __shared__ double red[GS_G][GS_C];
  __shared__ int acc_s[GS_C];
  const int cl = threadIdx.x % GS_C, rg = threadIdx.x / GS_C;
  const int64_t c = (int64_t)blockIdx.x * GS_C + cl;
  const bool in = c < k;
  double kk = 0.0, df = 0.0;
  if (in) {
    for (int64_t i = rg; i < n; i += GS_G) {
      const int64_t o = i * k + c;
      const double a = Atb[o], si = s[i];
      const double xn = Xn[o];
      const double g1 = HXn[o] - a, g0 = GX[o] - a;
      const double y = si * xn, gy = g1 / si;
      const double m = y < gy ? y : gy;
      kk += m * m;
      df += (xn - (double)X[o]) * (g0 + g1);
    }
  }
  kk = gs_reduce(kk, red, rg, cl);
  df = 0.5 * gs_reduce(df, red, rg, cl);
  if (in && rg == 0) {
    const double aa = colstat[c * 8 + 3];
    const double r1 = aa > 0.0 ? sqrt(kk) / sqrt(aa) : sqrt(kk);
    const double r0 = colstat[c * 8 + 0];
    const bool accept = (r1 < r0) && (df <= 0.0);
    acc_s[cl] = accept ? 1 : 0;
    kkt64[c] = accept ? r1 : r0;
  }
  __syncthreads();
  if (in && acc_s[cl])
    for (int64_t i = rg; i < n; i += GS_G) X[i * k + c] = (TX)Xn[i * k + c];
}

// F = 1/2 ||A X - B||^2 per column, from the residuals.  A 64 x 64 tile of R = A X - B (rows i of
// A, columns c of X) is summed over n on the FP64 matrix cores, as gemm_tn_f64_kernel sums over d,
// then squared and summed over its 64 rows: part[tile row][c].  resid_sq_reduce_kernel adds the
// row tiles in order.  Staging: A as sa[kk][i] (a thread loads column kk = tid % 32 of rows
// tid / 32 + 8 u), X as sx[kk][c] (column tid % 64 of rows tid / 64 + 4 u).
template <typename TA, typename TX>
__global__ __launch_bounds__(256, 4) void resid_sq_f64_kernel(int64_t d, int64_t n, int64_t k,
                                                              const TA* __restrict__ A,
                                                              int64_t lda,
                                                              const TX* __restrict__ X,
                                                              const TA* __restrict__ B,
                                                              int64_t ldb,
                                                              double* __restrict__ part) {
  __shared__ double sa[TN_BK][TN_LD];
  __shared__ double sx[TN_BK][TN_LD];
  __shared__ double colred[2][TN_T];
  const int64_t i0 = (int64_t)blockIdx.y * TN_T, c0 = (int64_t)blockIdx.x * TN_T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int ak = tid & 31, ar = tid >> 5;
  const int xc = tid & 63, xr = tid >> 6;
  TA ra[8];
  TX rx[8];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + ar + 8 * u, kk = k0 + ak;
      ra[u] = (i < d && kk < n) ? A[i * lda + kk] : (TA)0;
      const int64_t kx = k0 + xr + 4 * u, c = c0 + xc;
      rx[u] = (kx < n && c < k) ? X[kx * k + c] : (TX)0;
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const int col = lane & 15, kq = lane >> 4;
  load(0);
  for (int64_t k0 = 0; k0 < n; k0 += TN_BK) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sa[ak][ar + 8 * u] = (double)ra[u];
      sx[xr + 4 * u][xc] = (double)rx[u];
    }
    __syncthreads();
    if (k0 + TN_BK < n) load(k0 + TN_BK);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < TN_BK; kk += 4) {
      const int kr = kk + kq;
      const double a0 = sa[kr][wi + col], a1 = sa[kr][wi + 16 + col];
      const double b0 = sx[kr][wj + col], b1 = sx[kr][wj + 16 + col];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane l holds column l % 16 and rows l / 16 + 4 e of each 16 x 16 block
  double sq[2] = {0.0, 0.0};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int64_t c = c0 + wj + b * 16 + col;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = i0 + wi + a * 16 + kq + 4 * e;
        if (i < d && c < k) {
          const double r = acc[a][b][e] - (double)B[i * ldb + c];
          sq[b] += r * r;
        }
      }
    // the four row groups of a column (lanes col + 16 kq), in a fixed order
    sq[b] += __shfl_xor(sq[b], 16);
    sq[b] += __shfl_xor(sq[b], 32);
  }
  if (kq == 0) {
    colred[wave >> 1][wj + col] = sq[0];
    colred[wave >> 1][wj + 16 + col] = sq[1];
  }
  __syncthreads();
  if (tid < TN_T && c0 + tid < k)
    part[(int64_t)blockIdx.y * k + c0 + tid] = colred[0][tid] + colred[1][tid];
}

// obj64[c] = 1/2 * sum over the row tiles t of part[t][c], in order of t.
__global__ __launch_bounds__(256) void resid_sq_reduce_kernel(int64_t tiles, int64_t k,
                                                              const double* __restrict__ part,
                                                              double* __restrict__ obj64) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= k) return;
  double v = 0.0;
  for (int64_t t = 0; t < tiles; ++t) v += part[t * k + c];
  obj64[c] = 0.5 * v;
}

// ---- per-column steps ---------------------------------------------------------------------
// One workgroup of RS_NT threads per right-hand side: the few right-hand-side path has k <= 4
// columns, so each stage is a handful of workgroups whose time is the latency of their strided
// walks over d and n; 512 threads make those walks short (1024 would cap the registers at 128
// and spill).
constexpr int RS_NT = 512;

// sum over r < len of V[r * k + c]^2 by one thread, stride RS_NT from threadIdx.x, with eight
// loads in flight (the sums run in eight fixed lanes of accumulation, added in a fixed order).
__device__ __forceinline__ double strided_sumsq(const double* __restrict__ V, int64_t len,
                                                int64_t k, int64_t c) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t r = threadIdx.x;
  for (; r + 7 * RS_NT < len; r += 8 * RS_NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = V[(r + u * RS_NT) * k + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u] * v[u];
  }
  for (; r < len; r += RS_NT) {
    const double v = V[r * k + c];
    a[0] += v * v;
  }
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Stage 1 (after R, G, Atb, s): residual and objective at x, direction D = p ./ s, ||p||^2.
template <typename TX>
__global__ __launch_bounds__(RS_NT) void refine_stage1_kernel(int64_t d, int64_t n, int64_t k,
                                                            const TX* __restrict__ X,
                                                            const double* __restrict__ R,
                                                            const double* __restrict__ G,
                                                            const double* __restrict__ Atb,
                                                            const double* __restrict__ s,
                                                            double* __restrict__ D,
                                                            double* __restrict__ colstat) {
  __shared__ double red[RS_NT / 64];
  const int64_t c = blockIdx.x;
  double kk = 0.0, aa = 0.0, num = 0.0, ff = 0.0;
#pragma unroll 1
  for (int64_t i = threadIdx.x; i < n; i += RS_NT) {
    const double y = s[i] * (double)X[i * k + c];
    const double gy = G[i * k + c] / s[i];
    const bool pas = (y > 0.0) || (gy < 0.0);
    const double p = pas ? gy : 0.0;
    num += p * p;
    D[i * k + c] = p / s[i];
    const double m = y < gy ? y : gy;
    kk += m * m;
    const double ai = Atb[i * k + c] / s[i];
    aa += ai * ai;
  }
  ff = strided_sumsq(R, d, k, c);
  kk = block_sum<double, RS_NT>(kk, red);
  aa = block_sum<double, RS_NT>(aa, red);
  num = block_sum<double, RS_NT>(num, red);
  ff = block_sum<double, RS_NT>(ff, red);
  if (threadIdx.x == 0) {
    colstat[c * 8 + 0] = aa > 0.0 ? sqrt(kk) / sqrt(aa) : sqrt(kk);  // residual at x
    colstat[c * 8 + 1] = 0.5 * ff;                                  // objective at x
    colstat[c * 8 + 2] = num;
    colstat[c * 8 + 3] = aa;
  }
}

// Stage 2 (after V = A D): alpha and the candidate x'.
template <typename TX>
__global__ __launch_bounds__(RS_NT) void refine_stage2_kernel(int64_t d, int64_t n, int64_t k,
                                                            const TX* __restrict__ X,
                                                            const double* __restrict__ V,
                                                            const double* __restrict__ D,
                                                            double* __restrict__ Xn,
                                                            double* __restrict__ colstat) {
  __shared__ double red[RS_NT / 64];
  const int64_t c = blockIdx.x;
  double vv = strided_sumsq(V, d, k, c);
  vv = block_sum<double, RS_NT>(vv, red);
  const double num = colstat[c * 8 + 2];
  const double alpha = (vv > 0.0 && __builtin_isfinite(vv)) ? num / vv : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RS_NT) {
    const double v = (double)X[i * k + c] - alpha * D[i * k + c];
    // rounded to the output type here, so the residual reported for x' is that of the stored x'
    Xn[i * k + c] = (double)(TX)(v > 0.0 ? v : 0.0);
  }
  if (threadIdx.x == 0) colstat[c * 8 + 4] = alpha;
}

// Stage 3 (after R' = A x' - B, G' = A^T R'): accept or reject, write results.
template <typename TX>
__global__ __launch_bounds__(RS_NT) void refine_stage3_kernel(int64_t d, int64_t n, int64_t k,
                                                            TX* __restrict__ X,
                                                            const double* __restrict__ Xn,
                                                            const double* __restrict__ R2,
                                                            const double* __restrict__ G2,
                                                            const double* __restrict__ s,
                                                            const double* __restrict__ colstat,
                                                            double* __restrict__ kkt64,
                                                            double* __restrict__ obj64) {
  __shared__ double red[RS_NT / 64];
  const int64_t c = blockIdx.x;
  double ff = strided_sumsq(R2, d, k, c), kk = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RS_NT) {
    const double y = s[i] * Xn[i * k + c];
    const double gy = G2[i * k + c] / s[i];
    const double m = y < gy ? y : gy;
    kk += m * m;
  }
  ff = block_sum<double, RS_NT>(ff, red);
  kk = block_sum<double, RS_NT>(kk, red);
  const double F1 = 0.5 * ff;
  const double F0 = colstat[c * 8 + 1];
  const double aa = colstat[c * 8 + 3];
  const double r1 = aa > 0.0 ? sqrt(kk) / sqrt(aa) : sqrt(kk);
  const double r0 = colstat[c * 8 + 0];
  // The exact step lowers the objective along the masked gradient but, on an ill-conditioned
  // problem, can raise the KKT residual; keep it only when neither gets worse.
  const bool accept = (r1 < r0) && (F1 <= F0);
  if (accept) {
    for (int64_t i = threadIdx.x; i < n; i += RS_NT) X[i * k + c] = (TX)Xn[i * k + c];
  }
  if (threadIdx.x == 0) {
    kkt64[c] = accept ? r1 : r0;
    if (obj64 != nullptr) obj64[c] = accept ? F1 : F0;
  }
}

// ---- orchestration -------------------------------------------------------------------------
struct RefineWs {
  double *R, *V, *G, *Atb, *s, *D, *Xn, *colstat, *partial;
  int64_t chunks;
};

// Row chunks of the A^T V passes: enough workgroups to fill the GPU a few times over with
// 1024-column (vector path) or 256-column blocks; the partial sums cost chunks * n doubles.
static int64_t refine_chunks(int64_t d, int64_t n) {
  const int64_t bx = (n + 1023) / 1024;
  int64_t chunks = (768 + bx - 1) / bx;
  if (chunks > d) chunks = d;
  return chunks < 1 ? 1 : chunks;
}

static RefineWs refine_layout(void* ws, int64_t d, int64_t n, int64_t k) {
  RefineWs w;
  double* p = (double*)ws;
  w.R = p; p += d * k;
  w.V = p; p += d * k;
  w.G = p; p += n * k;
  w.Atb = p; p += n * k;
  w.s = p; p += n;
  w.D = p; p += n * k;
  w.Xn = p; p += n * k;
  w.colstat = p; p += 8 * k;
  w.chunks = refine_chunks(d, n);
  w.partial = p;
  return w;
}

// Gram path workspace: H [n, n], a, HX, D, HD (reused for H X'), X' [n, k], s [n],
// colstat [8 k], the row-tile sums of squared residuals [ceil(d / 64), k], and the partials of a
// split product.
struct GramRefineWs {
  double *H, *a, *HX, *D, *HD, *Xn, *s, *colstat, *rsq, *part;
};

static int64_t resid_tiles(int64_t d) { return (d + TN_T - 1) / TN_T; }

static GramRefineWs gram_refine_layout(void* ws, int64_t d, int64_t n, int64_t k) {
  GramRefineWs w;
  double* p = (double*)ws;
  w.H = p; p += n * n;
  w.a = p; p += n * k;
  w.HX = p; p += n * k;
  w.D = p; p += n * k;
  w.HD = p; p += n * k;
  w.Xn = p; p += n * k;
  w.s = p; p += n;
  w.colstat = p; p += 8 * k;
  w.rsq = p; p += resid_tiles(d) * k;
  w.part = p;
  return w;
}

static int gref_splits(int64_t d, int64_t n, int64_t k);

size_t refine_ws_bytes(int64_t d, int64_t n, int64_t k) {
  size_t el;
  if (k <= RF_SMALL_K) {
    // partial sums of the two-pass (chunks) or the fused (up to RC_MAX_WG workgroups) form
    const int64_t ch = refine_chunks(d, n) > RC_MAX_WG ? refine_chunks(d, n) : RC_MAX_WG;
    el = (size_t)(2 * d * k + 4 * n * k + n + 8 * k) + (size_t)ch * (2 * k + 1) * n;
  }
  else
    el = (size_t)(n * n + 5 * n * k + n + 8 * k) + (size_t)(resid_tiles(d) * k) +
         (size_t)gref_splits(d, n, k) * (size_t)(n * (n + k));
  return el * sizeof(double) + 256;
}

static bool vec_ok(const void* A, int64_t lda, int64_t n, size_t elem) {
  return elem == 4 && (lda % 4) == 0 && (n % 4) == 0 && (((uintptr_t)A) & 15) == 0;
}

template <typename T>
static void launch_resid(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda,
                         const void* X, bool x_is_double, const T* B, int64_t ldb, double* R,
                         hipStream_t st) {
  if (vec_ok(A, lda, n, sizeof(T))) {
    const int rpw = k == 1 ? RF_RPW1 : RF_RPW;
    dim3 grid((unsigned)((d + 4 * rpw - 1) / (4 * rpw)));
    const float* Af = (const float*)A;
    const float* Bf = (const float*)B;
    if (k == 1) {
      if (x_is_double)
        hipLaunchKernelGGL((rows_residual_vec_kernel<double, 1, RF_RPW1>), grid, dim3(256), 0, st,
                           d, n, k, Af, lda, (const double*)X, Bf, ldb, R);
      else
        hipLaunchKernelGGL((rows_residual_vec_kernel<float, 1, RF_RPW1>), grid, dim3(256), 0, st,
                           d, n, k, Af, lda, (const float*)X, Bf, ldb, R);
    } else {
      if (x_is_double)
        hipLaunchKernelGGL((rows_residual_vec_kernel<double, RF_SMALL_K, RF_RPW>), grid, dim3(256),
                           0, st, d, n, k, Af, lda, (const double*)X, Bf, ldb, R);
      else
        hipLaunchKernelGGL((rows_residual_vec_kernel<float, RF_SMALL_K, RF_RPW>), grid, dim3(256),
                           0, st, d, n, k, Af, lda, (const float*)X, Bf, ldb, R);
    }
  } else {
    dim3 grid((unsigned)((d + 3) / 4));
    if (x_is_double)
      hipLaunchKernelGGL((rows_residual_kernel<T, double>), grid, dim3(256), 0, st, d, n, k, A, lda,
                         (const double*)X, B, ldb, R);
    else
      hipLaunchKernelGGL((rows_residual_kernel<T, T>), grid, dim3(256), 0, st, d, n, k, A, lda,
                         (const T*)X, B, ldb, R);
  }
}

template <typename T>
static void launch_atr(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const double* R,
                       const T* B, int64_t ldb, bool with_b, RefineWs& w, double* G,
                       hipStream_t st) {
  const int64_t rows = (d + w.chunks - 1) / w.chunks;
  const int wb = with_b ? 1 : 0;
  if (vec_ok(A, lda, n, sizeof(T))) {
    dim3 g1((unsigned)((n + 1023) / 1024), (unsigned)w.chunks);
    const float* Af = (const float*)A;
    const float* Bf = (const float*)B;
    switch (k) {
#define CP_LAUNCH(KV)                                                                         \
  hipLaunchKernelGGL(cols_partial_vec_kernel<KV>, g1, dim3(256), 0, st, d, n, Af, lda, R, Bf, ldb, \
                     wb, rows, w.partial)
      case 1: CP_LAUNCH(1); break;
      case 2: CP_LAUNCH(2); break;
      case 3: CP_LAUNCH(3); break;
      default: CP_LAUNCH(4); break;
#undef CP_LAUNCH
    }
  } else {
    dim3 g1((unsigned)((n + 255) / 256), (unsigned)w.chunks);
    hipLaunchKernelGGL(cols_partial_kernel<T>, g1, dim3(256), 0, st, d, n, k, A, lda, R, B, ldb,
                       wb, rows, w.partial);
  }
  hipLaunchKernelGGL(cols_finalize_kernel, dim3((unsigned)((n + CF_C - 1) / CF_C)), dim3(256), 0,
                     st, n, k, wb, w.chunks, (const double*)w.partial, G, w.Atb, w.s);
}

static bool fused_ok(const void* A, int64_t lda, int64_t n, int64_t k, size_t elem) {
  return k == 1 && vec_ok(A, lda, n, elem) && n <= 2048 * RC_MAX_NB;
}

// R = A x - b and G = A^T R (with WB also A^T b and the column norms s) in one read of A.
template <typename TX>
static void launch_fused(int64_t d, int64_t n, const float* A, int64_t lda, const TX* X,
                         const float* B, int64_t ldb, bool with_b, RefineWs& w, double* R,
                         double* G, hipStream_t st) {
  // contiguous row ranges, a multiple of 4 rows each (so of every step size)
  int64_t grid = (d + 3) / 4;
  if (grid > RC_MAX_WG) grid = RC_MAX_WG;
  int64_t rows = (d + grid - 1) / grid;
  rows = (rows + 3) / 4 * 4;
  grid = (d + rows - 1) / rows;
  const int nb = (int)((n + 2047) / 2048);
  dim3 g((unsigned)grid), b(RC_NT);
#define RC_LAUNCH(NB, WB)                                                                       \
  hipLaunchKernelGGL((rows_cols_fused_kernel<NB, WB, TX>), g, b, 0, st, d, n, A, lda, X, B, ldb, \
                     rows, R, w.partial)
  if (with_b) {
    if (nb == 1) RC_LAUNCH(1, true);
    else if (nb == 2) RC_LAUNCH(2, true);
    else RC_LAUNCH(3, true);
  } else {
    if (nb == 1) RC_LAUNCH(1, false);
    else if (nb == 2) RC_LAUNCH(2, false);
    else RC_LAUNCH(3, false);
  }
#undef RC_LAUNCH
  hipLaunchKernelGGL(cols_finalize_kernel, dim3((unsigned)((n + CF_C - 1) / CF_C)), dim3(256), 0,
                     st, n, (int64_t)1, with_b ? 1 : 0, grid, (const double*)w.partial, G, w.Atb,
                     w.s);
}

// C = A^T [M1 | M2] (see gemm_tn_f64_kernel).  S > 1 splits the sum over K into S row ranges
// with partials in part (S N (n1 + n2) doubles), added by a second kernel.
template <typename TA, typename TM>
static void gemm_tn(int64_t K, int64_t N, const TA* A, int64_t lda, int64_t n1, const TM* M1,
                    int64_t ld1, double* C1, int64_t ldc1, int64_t n2, const TM* M2, int64_t ld2,
                    double* C2, int64_t ldc2, hipStream_t st, int S = 1,
                    double* part = nullptr) {
  if (S <= 1) part = nullptr;
  const int64_t kps = part ? ((K + S - 1) / S + TN_BK - 1) / TN_BK * TN_BK : K;
  dim3 grid((unsigned)((n1 + n2 + TN_T - 1) / TN_T), (unsigned)((N + TN_T - 1) / TN_T),
            part ? (unsigned)S : 1u);
  hipLaunchKernelGGL((gemm_tn_f64_kernel<TA, TM>), grid, dim3(256), 0, st, K, N, n1, n2, A, lda,
                     M1, ld1, M2, ld2, C1, ldc1, C2, ldc2, kps, part);
  if (part) {
    const int64_t tot = N * (n1 + n2);
    hipLaunchKernelGGL(gemm_tn_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                       st, S, N, n1, n2, (const double*)part, C1, ldc1, C2, ldc2);
  }
}

// K splits of the FP64 Gram [A | B]^T A.  With fewer than two 64 x 64 tiles per compute unit
// the busiest unit does ceil(tiles / CUs) tiles; splitting K S ways makes that
// ceil(tiles S / CUs) / S tiles' worth.  S minimises that plus 1 % per split (the partials), at
// most 8 splits of at least 256 rows each.
static int gref_splits(int64_t d, int64_t n, int64_t k) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t tiles = ((n + k + TN_T - 1) / TN_T) * ((n + TN_T - 1) / TN_T);
  if (cus < 1 || tiles >= 2 * (int64_t)cus) return 1;
  int best = 1;
  double best_cost = 1e30;
  for (int S = 1; S <= 8 && (S == 1 || (int64_t)S * 256 <= d); ++S) {
    const double cost = (double)((tiles * S + cus - 1) / cus) / S + 0.01 * S;
    if (cost < best_cost) {
      best_cost = cost;
      best = S;
    }
  }
  return best;
}

template <typename T>
static void launch_refine_gram(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda,
                               const T* B, int64_t ldb, T* X, double* kkt64, double* obj64,
                               void* ws, hipStream_t st) {
  GramRefineWs w = gram_refine_layout(ws, d, n, k);
  const unsigned cb = (unsigned)((k + GS_C - 1) / GS_C);
  // H = A^T A and a = A^T B in one launch over the columns of [A | B]
  gemm_tn<T, T>(d, n, A, lda, n, A, lda, w.H, n, k, B, ldb, w.a, k, st, gref_splits(d, n, k),
                w.part);
  hipLaunchKernelGGL(diag_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                     (const double*)w.H, w.s);
  // H is symmetric, so H^T M = H M: the same transposed product with K = n
  gemm_tn<double, T>(n, n, w.H, n, k, X, k, w.HX, k, 0, (const T*)nullptr, 0, nullptr, 0, st);
  hipLaunchKernelGGL(gref_stage1_kernel<T>, dim3(cb), dim3(256), 0, st, n, k, (const T*)X,
                     (const double*)w.HX, (const double*)w.a, (const double*)w.s, w.D,
                     w.colstat);
  gemm_tn<double, double>(n, n, w.H, n, k, w.D, k, w.HD, k, 0, (const double*)nullptr, 0,
                          nullptr, 0, st);
  hipLaunchKernelGGL(gref_stage2_kernel<T>, dim3(cb), dim3(256), 0, st, n, k, (const T*)X,
                     (const double*)w.D, (const double*)w.HD, w.Xn, (const double*)w.colstat);
  gemm_tn<double, double>(n, n, w.H, n, k, w.Xn, k, w.HD, k, 0, (const double*)nullptr, 0,
                          nullptr, 0, st);  // H x' (reuses HD)
  hipLaunchKernelGGL(gref_stage3_kernel<T>, dim3(cb), dim3(256), 0, st, n, k, X,
                     (const double*)w.Xn, (const double*)w.HD, (const double*)w.HX,
                     (const double*)w.a, (const double*)w.s, (const double*)w.colstat, kkt64);
  if (obj64 != nullptr) {
    // F of the returned X from its residuals
    const int64_t tiles = resid_tiles(d);
    dim3 g((unsigned)((k + TN_T - 1) / TN_T), (unsigned)tiles);
    hipLaunchKernelGGL((resid_sq_f64_kernel<T, T>), g, dim3(256), 0, st, d, n, k, A, lda,
                       (const T*)X, B, ldb, w.rsq);
    hipLaunchKernelGGL(resid_sq_reduce_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0,
                       st, tiles, k, (const double*)w.rsq, obj64);
  }
}

template <typename T>
hipError_t launch_refine(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
                         int64_t ldb, T* X, double* kkt64, double* obj64, void* ws,
                         hipStream_t st) {
  if (k > RF_SMALL_K) {
    launch_refine_gram<T>(d, n, k, A, lda, B, ldb, X, kkt64, obj64, ws, st);
    return hipGetLastError();
  }
  RefineWs w = refine_layout(ws, d, n, k);
  const bool fused = fused_ok(A, lda, n, k, sizeof(T));
  if (fused) {
    launch_fused<T>(d, n, (const float*)A, lda, (const T*)X, (const float*)B, ldb, true, w, w.R,
                    w.G, st);
  } else {
    launch_resid<T>(d, n, k, A, lda, X, false, B, ldb, w.R, st);
    launch_atr<T>(d, n, k, A, lda, w.R, B, ldb, true, w, w.G, st);
  }
  hipLaunchKernelGGL(refine_stage1_kernel<T>, dim3((unsigned)k), dim3(RS_NT), 0, st, d, n, k,
                     (const T*)X, (const double*)w.R, (const double*)w.G, (const double*)w.Atb,
                     (const double*)w.s, w.D, w.colstat);
  launch_resid<T>(d, n, k, A, lda, w.D, true, (const T*)nullptr, 0, w.V, st);
  hipLaunchKernelGGL(refine_stage2_kernel<T>, dim3((unsigned)k), dim3(RS_NT), 0, st, d, n, k,
                     (const T*)X, (const double*)w.V, (const double*)w.D, w.Xn, w.colstat);
  if (fused) {
    launch_fused<double>(d, n, (const float*)A, lda, (const double*)w.Xn, (const float*)B, ldb,
                         false, w, w.R, w.G, st);
  } else {
    launch_resid<T>(d, n, k, A, lda, w.Xn, true, B, ldb, w.R, st);
    launch_atr<T>(d, n, k, A, lda, w.R, B, ldb, false, w, w.G, st);
  }
  hipLaunchKernelGGL(refine_stage3_kernel<T>, dim3((unsigned)k), dim3(RS_NT), 0, st, d, n, k, X,
                     (const double*)w.Xn, (const double*)w.R, (const double*)w.G,
                     (const double*)w.s, (const double*)w.colstat, kkt64, obj64);
  return hipGetLastError();
}
template hipError_t launch_refine<float>(int64_t, int64_t, int64_t, const float*, int64_t,
                                        const float*, int64_t, float*, double*, double*, void*,
                                        hipStream_t);
template hipError_t launch_refine<double>(int64_t, int64_t, int64_t, const double*, int64_t,
                                         const double*, int64_t, double*, double*, double*, void*,
                                         hipStream_t);

}  // namespace nnls
