// FP64 check and one refinement step against the original data (A, B).
//
// Products with A are done in FP64 arithmetic on the stored entries of A (FP32 or FP64):
//   R = A X - B,  G = A^T R,  a = A^T B,  s_i^2 = sum_r A_ri^2           (passes 1 and 2)
//   in the rescaled variables y = s .* x, grad_y = G ./ s: passive set, masked gradient p,
//   relative KKT residual ||min(y, grad_y)|| / ||a ./ s||                 (per column)
//   V = A (p ./ s), alpha = ||p||^2 / ||V||^2  (= p^T Q p in exact arithmetic) (pass 3)
//   x' = [x - alpha p ./ s]_+, R' = A x' - B, G' = A^T R'                   (passes 4 and 5)
//   keep x' when it lowers the residual without raising 1/2||A x - b||^2, and report the
//   residual and objective of the x that is returned.
// Few right-hand sides use matrix-vector kernels that stream A once per pass; many use a
// tiled FP64 product.
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
// wave takes RF_RPW rows at once, each lane 4 consecutive columns per step, so one load of x
// serves RF_RPW rows and RF_RPW independent 16-byte loads of A are in flight per step.
constexpr int RF_RPW = 4;

template <typename TX>
__device__ __forceinline__ void load_x4(const TX* X, int64_t i, int64_t k, int c, double* xv) {
#pragma unroll
  for (int e = 0; e < 4; ++e) xv[e] = (double)X[(i + e) * k + c];
}

template <typename TX>
__global__ __launch_bounds__(256) void rows_residual_vec_kernel(int64_t d, int64_t n, int64_t k,
                                                                const float* __restrict__ A,
                                                                int64_t lda,
                                                                const TX* __restrict__ X,
                                                                const float* __restrict__ B,
                                                                int64_t ldb,
                                                                double* __restrict__ R) {
  const int lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RF_RPW;
  if (r0 >= d) return;
  double acc[RF_RPW][RF_SMALL_K];
#pragma unroll
  for (int q = 0; q < RF_RPW; ++q)
#pragma unroll
    for (int c = 0; c < RF_SMALL_K; ++c) acc[q][c] = 0.0;
  for (int64_t i = 4 * lane; i < n; i += 256) {
    f32x4 a[RF_RPW];
#pragma unroll
    for (int q = 0; q < RF_RPW; ++q)
      a[q] = (r0 + q < d) ? *(const f32x4*)(A + (r0 + q) * lda + i) : (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < RF_SMALL_K; ++c) {
      if (c < k) {
        double xv[4];
        load_x4(X, i, k, c, xv);
#pragma unroll
        for (int q = 0; q < RF_RPW; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[q][c] += (double)a[q][e] * xv[e];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RF_RPW; ++q) {
#pragma unroll
    for (int c = 0; c < RF_SMALL_K; ++c) {
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

__global__ __launch_bounds__(256) void cols_finalize_kernel(int64_t n, int64_t k, int with_b,
                                                            int64_t nchunks,
                                                            const double* __restrict__ partial,
                                                            double* __restrict__ G,
                                                            double* __restrict__ Atb,
                                                            double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int nvec = with_b ? (int)(2 * k + 1) : (int)k;
  for (int m = 0; m < nvec; ++m) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t c = 0;
    for (; c + 3 < nchunks; c += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += partial[((c + u) * nvec + m) * n + i];
    }
    for (; c < nchunks; ++c) a[0] += partial[(c * nvec + m) * n + i];
    const double acc = (a[0] + a[1]) + (a[2] + a[3]);
    if (m < k) G[i * k + m] = acc;
    else if (m < 2 * k) Atb[i * k + (m - k)] = acc;
    else s[i] = acc > 0.0 ? sqrt(acc) : 1.0;
  }
}

// ---- many right-hand sides: tiled FP64 products -----------------------------------------------
// TRANS = false: C[M, N] = A[M, K] * Bm[K, N] - Cin      (A row-major [d, n], M = d, K = n)
// TRANS = true:  C[M, N] = A^T[M, K] * Bm[K, N]           (A row-major [d, n], M = n, K = d)
// Bm is FP64 [K, N] with leading dimension ldbm; Cin (optional, element type TA) is subtracted.
// When with_sq, column sums of squares of A are also produced (TRANS only, tile column 0).
constexpr int RG_BM = 64;
constexpr int RG_BK = 16;

template <typename TA, typename TB, bool TRANS>
__global__ __launch_bounds__(256) void gemm64_kernel(int64_t M, int64_t N, int64_t K,
                                                     const TA* __restrict__ A, int64_t lda,
                                                     const TB* __restrict__ Bm, int64_t ldbm,
                                                     const TA* __restrict__ Cin, int64_t ldcin,
                                                     double* __restrict__ C, int64_t ldc) {
  __shared__ double sa[RG_BK][RG_BM + 1];
  __shared__ double sb[RG_BK][RG_BM + 1];
  const int64_t m0 = (int64_t)blockIdx.y * RG_BM, n0 = (int64_t)blockIdx.x * RG_BM;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t k0 = 0; k0 < K; k0 += RG_BK) {
    for (int e = threadIdx.x; e < RG_BK * RG_BM; e += 256) {
      int kk, mm;
      if (TRANS) {  // A^T[m, k] = A[k, m]: consecutive threads along m (contiguous in A)
        kk = e / RG_BM;
        mm = e % RG_BM;
      } else {      // A[m, k]: consecutive threads along k
        mm = e / RG_BK;
        kk = e % RG_BK;
      }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < M && gk < K) v = TRANS ? (double)A[gk * lda + gm] : (double)A[gm * lda + gk];
      sa[kk][mm] = v;
      const int bk = e / RG_BM, bn = e % RG_BM;
      const int64_t gbk = k0 + bk, gbn = n0 + bn;
      sb[bk][bn] = (gbk < K && gbn < N) ? (double)Bm[gbk * ldbm + gbn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RG_BK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sa[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sb[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t gm = m0 + ty + 16 * a, gn = n0 + tx + 16 * b;
      if (gm < M && gn < N) {
        double v = acc[a][b];
        if (Cin) v -= (double)Cin[gm * ldcin + gn];
        C[gm * ldc + gn] = v;
      }
    }
}

// Column sums of squares of A (FP64), for the many-RHS path.
template <typename TA>
__global__ __launch_bounds__(256) void sumsq_cols_kernel(int64_t d, int64_t n,
                                                         const TA* __restrict__ A, int64_t lda,
                                                         double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t r = 0; r < d; ++r) {
    const double a = (double)A[r * lda + i];
    acc += a * a;
  }
  s[i] = acc > 0.0 ? sqrt(acc) : 1.0;
}

// ---- per-column steps ---------------------------------------------------------------------
// Stage 1 (after R, G, Atb, s): residual and objective at x, direction D = p ./ s, ||p||^2.
template <typename TX>
__global__ __launch_bounds__(256) void refine_stage1_kernel(int64_t d, int64_t n, int64_t k,
                                                            const TX* __restrict__ X,
                                                            const double* __restrict__ R,
                                                            const double* __restrict__ G,
                                                            const double* __restrict__ Atb,
                                                            const double* __restrict__ s,
                                                            double* __restrict__ D,
                                                            double* __restrict__ colstat) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double kk = 0.0, aa = 0.0, num = 0.0, ff = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
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
  for (int64_t r = threadIdx.x; r < d; r += 256) {
    const double v = R[r * k + c];
    ff += v * v;
  }
  kk = block_sum<double, 256>(kk, red);
  aa = block_sum<double, 256>(aa, red);
  num = block_sum<double, 256>(num, red);
  ff = block_sum<double, 256>(ff, red);
  if (threadIdx.x == 0) {
    colstat[c * 8 + 0] = aa > 0.0 ? sqrt(kk) / sqrt(aa) : sqrt(kk);  // residual at x
    colstat[c * 8 + 1] = 0.5 * ff;                                  // objective at x
    colstat[c * 8 + 2] = num;
    colstat[c * 8 + 3] = aa;
  }
}

// Stage 2 (after V = A D): alpha and the candidate x'.
template <typename TX>
__global__ __launch_bounds__(256) void refine_stage2_kernel(int64_t d, int64_t n, int64_t k,
                                                            const TX* __restrict__ X,
                                                            const double* __restrict__ V,
                                                            const double* __restrict__ D,
                                                            double* __restrict__ Xn,
                                                            double* __restrict__ colstat) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double vv = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += 256) {
    const double v = V[r * k + c];
    vv += v * v;
  }
  vv = block_sum<double, 256>(vv, red);
  const double num = colstat[c * 8 + 2];
  const double alpha = (vv > 0.0 && __builtin_isfinite(vv)) ? num / vv : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = (double)X[i * k + c] - alpha * D[i * k + c];
    // rounded to the output type here, so the residual reported for x' is that of the stored x'
    Xn[i * k + c] = (double)(TX)(v > 0.0 ? v : 0.0);
  }
  if (threadIdx.x == 0) colstat[c * 8 + 4] = alpha;
}

// Stage 3 (after R' = A x' - B, G' = A^T R'): accept or reject, write results.
template <typename TX>
__global__ __launch_bounds__(256) void refine_stage3_kernel(int64_t d, int64_t n, int64_t k,
                                                            TX* __restrict__ X,
                                                            const double* __restrict__ Xn,
                                                            const double* __restrict__ R2,
                                                            const double* __restrict__ G2,
                                                            const double* __restrict__ s,
                                                            const double* __restrict__ colstat,
                                                            double* __restrict__ kkt64,
                                                            double* __restrict__ obj64) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double ff = 0.0, kk = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += 256) {
    const double v = R2[r * k + c];
    ff += v * v;
  }
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double y = s[i] * Xn[i * k + c];
    const double gy = G2[i * k + c] / s[i];
    const double m = y < gy ? y : gy;
    kk += m * m;
  }
  ff = block_sum<double, 256>(ff, red);
  kk = block_sum<double, 256>(kk, red);
  const double F1 = 0.5 * ff;
  const double F0 = colstat[c * 8 + 1];
  const double aa = colstat[c * 8 + 3];
  const double r1 = aa > 0.0 ? sqrt(kk) / sqrt(aa) : sqrt(kk);
  const double r0 = colstat[c * 8 + 0];
  // The exact step lowers the objective along the masked gradient but, on an ill-conditioned
  // problem, can raise the KKT residual; keep it only when neither gets worse.
  const bool accept = (r1 < r0) && (F1 <= F0);
  if (accept) {
    for (int64_t i = threadIdx.x; i < n; i += 256) X[i * k + c] = (TX)Xn[i * k + c];
  }
  if (threadIdx.x == 0) {
    kkt64[c] = accept ? r1 : r0;
    obj64[c] = accept ? F1 : F0;
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

size_t refine_ws_bytes(int64_t d, int64_t n, int64_t k) {
  size_t el = (size_t)(2 * d * k + 4 * n * k + n + 8 * k);
  if (k <= RF_SMALL_K) el += (size_t)refine_chunks(d, n) * (2 * k + 1) * n;
  return el * sizeof(double) + 256;
}

static bool vec_ok(const void* A, int64_t lda, int64_t n, size_t elem) {
  return elem == 4 && (lda % 4) == 0 && (n % 4) == 0 && (((uintptr_t)A) & 15) == 0;
}

template <typename T>
static void launch_resid(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda,
                         const void* X, bool x_is_double, const T* B, int64_t ldb, double* R,
                         hipStream_t st) {
  if (k <= RF_SMALL_K && vec_ok(A, lda, n, sizeof(T))) {
    dim3 grid((unsigned)((d + 4 * RF_RPW - 1) / (4 * RF_RPW)));
    if (x_is_double)
      hipLaunchKernelGGL(rows_residual_vec_kernel<double>, grid, dim3(256), 0, st, d, n, k,
                         (const float*)A, lda, (const double*)X, (const float*)B, ldb, R);
    else
      hipLaunchKernelGGL(rows_residual_vec_kernel<float>, grid, dim3(256), 0, st, d, n, k,
                         (const float*)A, lda, (const float*)X, (const float*)B, ldb, R);
  } else if (k <= RF_SMALL_K) {
    dim3 grid((unsigned)((d + 3) / 4));
    if (x_is_double)
      hipLaunchKernelGGL((rows_residual_kernel<T, double>), grid, dim3(256), 0, st, d, n, k, A, lda,
                         (const double*)X, B, ldb, R);
    else
      hipLaunchKernelGGL((rows_residual_kernel<T, T>), grid, dim3(256), 0, st, d, n, k, A, lda,
                         (const T*)X, B, ldb, R);
  } else {
    dim3 grid((unsigned)((k + RG_BM - 1) / RG_BM), (unsigned)((d + RG_BM - 1) / RG_BM));
    if (x_is_double)
      hipLaunchKernelGGL((gemm64_kernel<T, double, false>), grid, dim3(256), 0, st, d, k, n, A, lda,
                         (const double*)X, k, B, ldb, R, k);
    else
      hipLaunchKernelGGL((gemm64_kernel<T, T, false>), grid, dim3(256), 0, st, d, k, n, A, lda,
                         (const T*)X, k, B, ldb, R, k);
  }
}

template <typename T>
static void launch_atr(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const double* R,
                       const T* B, int64_t ldb, bool with_b, RefineWs& w, double* G,
                       hipStream_t st) {
  if (k <= RF_SMALL_K && vec_ok(A, lda, n, sizeof(T))) {
    const int64_t rows = (d + w.chunks - 1) / w.chunks;
    dim3 g1((unsigned)((n + 1023) / 1024), (unsigned)w.chunks);
    const float* Af = (const float*)A;
    const float* Bf = (const float*)B;
    const int wb = with_b ? 1 : 0;
    switch (k) {
      case 1: hipLaunchKernelGGL(cols_partial_vec_kernel<1>, g1, dim3(256), 0, st, d, n, Af, lda, R, Bf, ldb, wb, rows, w.partial); break;
      case 2: hipLaunchKernelGGL(cols_partial_vec_kernel<2>, g1, dim3(256), 0, st, d, n, Af, lda, R, Bf, ldb, wb, rows, w.partial); break;
      case 3: hipLaunchKernelGGL(cols_partial_vec_kernel<3>, g1, dim3(256), 0, st, d, n, Af, lda, R, Bf, ldb, wb, rows, w.partial); break;
      default: hipLaunchKernelGGL(cols_partial_vec_kernel<4>, g1, dim3(256), 0, st, d, n, Af, lda, R, Bf, ldb, wb, rows, w.partial); break;
    }
    hipLaunchKernelGGL(cols_finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       k, wb, w.chunks, (const double*)w.partial, G, w.Atb, w.s);
  } else if (k <= RF_SMALL_K) {
    const int64_t rows = (d + w.chunks - 1) / w.chunks;
    dim3 g1((unsigned)((n + 255) / 256), (unsigned)w.chunks);
    hipLaunchKernelGGL(cols_partial_kernel<T>, g1, dim3(256), 0, st, d, n, k, A, lda, R, B, ldb,
                       with_b ? 1 : 0, rows, w.partial);
    hipLaunchKernelGGL(cols_finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       k, with_b ? 1 : 0, w.chunks, (const double*)w.partial, G, w.Atb, w.s);
  } else {
    dim3 grid((unsigned)((k + RG_BM - 1) / RG_BM), (unsigned)((n + RG_BM - 1) / RG_BM));
    hipLaunchKernelGGL((gemm64_kernel<T, double, true>), grid, dim3(256), 0, st, n, k, d, A, lda, R,
                       k, (const T*)nullptr, 0, G, k);
    if (with_b) {
      // a = A^T B: the same product with B (element type T) as the right operand.
      hipLaunchKernelGGL((gemm64_kernel<T, T, true>), grid, dim3(256), 0, st, n, k, d, A, lda, B,
                         ldb, (const T*)nullptr, 0, w.Atb, k);
      hipLaunchKernelGGL(sumsq_cols_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                         d, n, A, lda, w.s);
    }
  }
}

template <typename T>
hipError_t launch_refine(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
                         int64_t ldb, T* X, double* kkt64, double* obj64, void* ws,
                         hipStream_t st) {
  RefineWs w = refine_layout(ws, d, n, k);
  launch_resid<T>(d, n, k, A, lda, X, false, B, ldb, w.R, st);
  launch_atr<T>(d, n, k, A, lda, w.R, B, ldb, true, w, w.G, st);
  hipLaunchKernelGGL(refine_stage1_kernel<T>, dim3((unsigned)k), dim3(256), 0, st, d, n, k,
                     (const T*)X, (const double*)w.R, (const double*)w.G, (const double*)w.Atb,
                     (const double*)w.s, w.D, w.colstat);
  launch_resid<T>(d, n, k, A, lda, w.D, true, (const T*)nullptr, 0, w.V, st);
  hipLaunchKernelGGL(refine_stage2_kernel<T>, dim3((unsigned)k), dim3(256), 0, st, d, n, k,
                     (const T*)X, (const double*)w.V, (const double*)w.D, w.Xn, w.colstat);
  launch_resid<T>(d, n, k, A, lda, w.Xn, true, B, ldb, w.R, st);
  launch_atr<T>(d, n, k, A, lda, w.R, B, ldb, false, w, w.G, st);
  hipLaunchKernelGGL(refine_stage3_kernel<T>, dim3((unsigned)k), dim3(256), 0, st, d, n, k, X,
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
