// Gram product and rescale of Algorithm 1 (Problem (2) -> Problem (5)) for gfx950.
//
//   colnorm     s_i = ||A_i||_2 in FP64 from the stored entries (1 for a zero column)
//   gram_bf16x3 upper-triangle tiles of [A | B]^T [A | B] restricted to rows of A, so one launch
//               gives H = A^T A and A^T B.  FP32 inputs are split into hi + lo bfloat16 while
//               they are staged into LDS; each tile accumulates hi*hi + hi*lo + lo*hi on the
//               matrix cores (v_mfma_f32_16x16x32_bf16) in FP32.  The epilogue applies the
//               rescale of Problem (5) directly: Q_ij = H_ij / (s_i s_j), Q_ii = 1, q = -A^T B / s,
//               and mirrors the tile into the lower triangle.
//   gram_fma    the same product with plain FMAs in FP32 or FP64 (FP64 problems and the FP32
//               accuracy cross-check).
// Split-K over the rows of A is available for shapes with few output tiles; the partial tiles
// then go through gram_splitk_epilogue.
#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

// ---------------------------------------------------------------------------------------------
// Column norms in FP64: partial sums over row chunks, then a fixed-order reduction.
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void colnorm_partial_kernel(int64_t d, int64_t n, const T* A,
                                                              int64_t lda, int64_t rows_per_chunk,
                                                              double* partial) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (col >= n) return;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < d ? r0 + rows_per_chunk : d;
  double acc0 = 0.0, acc1 = 0.0;
  int64_t r = r0;
  for (; r + 1 < r1; r += 2) {
    double a = (double)A[r * lda + col];
    double b = (double)A[(r + 1) * lda + col];
    acc0 += a * a;
    acc1 += b * b;
  }
  if (r < r1) {
    double a = (double)A[r * lda + col];
    acc0 += a * a;
  }
  partial[chunk * n + col] = acc0 + acc1;
}

__global__ __launch_bounds__(256) void colnorm_finalize_kernel(int64_t n, int64_t nchunks,
                                                               const double* partial, double* s) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= n) return;
  double acc = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) acc += partial[c * n + col];
  s[col] = acc > 0.0 ? sqrt(acc) : 1.0;
}

// ---------------------------------------------------------------------------------------------
// Epilogue shared by all Gram variants: one entry (i, j) of [A | B]^T [A | B] with i < n.
// ---------------------------------------------------------------------------------------------
// Q is written from one computed value per unordered pair {i, j}, so it is exactly symmetric:
// tiles above the diagonal mirror every entry; in diagonal tiles only i <= j is emitted.
template <typename T, typename Acc>
__device__ __forceinline__ void gram_emit(int64_t i, int64_t j, Acc val, int64_t n, int64_t k,
                                          const double* __restrict__ s, T* __restrict__ Q,
                                          T* __restrict__ q, bool diag_tile) {
  if (i >= n) return;
  if (j < n) {
    if (diag_tile && i > j) return;
    T out;
    if (i == j) {
      out = val > (Acc)0 ? (T)1 : (T)0;
    } else {
      out = (T)((double)val / (s[i] * s[j]));
    }
    Q[i * n + j] = out;
    if (i != j) Q[j * n + i] = out;
  } else if (j < n + k) {
    q[i * k + (j - n)] = (T)(-(double)val / s[i]);
  }
}

// Tile index -> (ti, tj) with ti < tiles_a (rows of A) and ti <= tj < tiles_aug.
__device__ __forceinline__ void decode_tile(int tile, int tiles_aug, int& ti, int& tj) {
  int t = 0, rem = tile;
  while (rem >= tiles_aug - t) {
    rem -= tiles_aug - t;
    ++t;
  }
  ti = t;
  tj = t + rem;
}

// ---------------------------------------------------------------------------------------------
// BF16x3 Gram on the matrix cores.  128 x 128 tile per workgroup of 4 waves (2 x 2 waves of
// 64 x 64), K staged 32 rows at a time.  LDS holds hi and lo parts of both panels, column-major
// (32 consecutive k of one column contiguous, rows padded to 40 bf16 = 80 bytes so that the
// 16-byte accesses of 16 consecutive lanes hit distinct banks).
// ---------------------------------------------------------------------------------------------
constexpr int GB_BM = 128;
constexpr int GB_BK = 32;
constexpr int GB_LDK = 40;  // padded k stride in bf16 units

struct GramPanelPtr {
  const float* base;
  int64_t ld;
};

__device__ __forceinline__ GramPanelPtr panel_column(int64_t col, int64_t n, int64_t k,
                                                     const float* A, int64_t lda, const float* B,
                                                     int64_t ldb) {
  GramPanelPtr p;
  if (col < n) {
    p.base = A + col;
    p.ld = lda;
  } else if (col < n + k) {
    p.base = B + (col - n);
    p.ld = ldb;
  } else {
    p.base = nullptr;
    p.ld = 0;
  }
  return p;
}

__global__ __launch_bounds__(256) void gram_bf16x3_kernel(
    int64_t d, int64_t n, int64_t k, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, const double* __restrict__ s, float* __restrict__ Q,
    float* __restrict__ q, float* __restrict__ partial, int tiles_aug, int64_t rows_per_split) {
  __shared__ __attribute__((aligned(16))) uint16_t sXh[GB_BM * GB_LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sXl[GB_BM * GB_LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sYh[GB_BM * GB_LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sYl[GB_BM * GB_LDK];

  int ti, tj;
  decode_tile(blockIdx.x, tiles_aug, ti, tj);
  const bool diag = (ti == tj);
  const int64_t i0 = (int64_t)ti * GB_BM, j0 = (int64_t)tj * GB_BM;
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r_end = r_begin + rows_per_split < d ? r_begin + rows_per_split : d;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lc = tid & 127;     // column of the panel this thread stages
  const int kh = tid >> 7;      // which 16-row half of the K chunk

  const GramPanelPtr px = panel_column(i0 + lc, n, k, A, lda, B, ldb);
  const GramPanelPtr py = panel_column(j0 + lc, n, k, A, lda, B, ldb);

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

  float rx[16], ry[16];
  auto load_chunk = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t r = r0 + kh * 16 + u;
      const bool ok = r < r_end;
      rx[u] = (ok && px.base) ? px.base[r * px.ld] : 0.f;
      ry[u] = (!diag && ok && py.base) ? py.base[r * py.ld] : 0.f;
    }
  };
  auto store_chunk = [&]() {
    uint32_t hx[8], lx[8], hy[8], ly[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      uint32_t h0, l0, h1, l1;
      split_bf16(rx[2 * u], h0, l0);
      split_bf16(rx[2 * u + 1], h1, l1);
      hx[u] = h0 | (h1 << 16);
      lx[u] = l0 | (l1 << 16);
      if (!diag) {
        split_bf16(ry[2 * u], h0, l0);
        split_bf16(ry[2 * u + 1], h1, l1);
        hy[u] = h0 | (h1 << 16);
        ly[u] = l0 | (l1 << 16);
      }
    }
    const int off = lc * GB_LDK + kh * 16;
    *(u32x4*)&sXh[off] = (u32x4){hx[0], hx[1], hx[2], hx[3]};
    *(u32x4*)&sXh[off + 8] = (u32x4){hx[4], hx[5], hx[6], hx[7]};
    *(u32x4*)&sXl[off] = (u32x4){lx[0], lx[1], lx[2], lx[3]};
    *(u32x4*)&sXl[off + 8] = (u32x4){lx[4], lx[5], lx[6], lx[7]};
    if (!diag) {
      *(u32x4*)&sYh[off] = (u32x4){hy[0], hy[1], hy[2], hy[3]};
      *(u32x4*)&sYh[off + 8] = (u32x4){hy[4], hy[5], hy[6], hy[7]};
      *(u32x4*)&sYl[off] = (u32x4){ly[0], ly[1], ly[2], ly[3]};
      *(u32x4*)&sYl[off + 8] = (u32x4){ly[4], ly[5], ly[6], ly[7]};
    }
  };

  const uint16_t* yh = diag ? sXh : sYh;
  const uint16_t* yl = diag ? sXl : sYl;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const int frag_row = lane & 15;
  const int frag_k = (lane >> 4) * 8;

  if (r_begin < r_end) load_chunk(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += GB_BK) {
    __syncthreads();  // previous chunk fully consumed
    store_chunk();
    __syncthreads();
    if (r0 + GB_BK < r_end) load_chunk(r0 + GB_BK);  // prefetch overlaps the MFMAs below

    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int xo = (wm + t * 16 + frag_row) * GB_LDK + frag_k;
      const int yo = (wn + t * 16 + frag_row) * GB_LDK + frag_k;
      ah[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&sXh[xo]);
      al[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&sXl[xo]);
      bh[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&yh[yo]);
      bl[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&yl[yo]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
      }
  }

  // D fragment layout of the 16x16 MFMA: lane holds column (lane & 15), rows 4*(lane>>4)+e.
  const int out_col = lane & 15;
  const int out_row = (lane >> 4) * 4;
  if (partial == nullptr) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t i = i0 + wm + a * 16 + out_row + e;
          const int64_t j = j0 + wn + b * 16 + out_col;
          gram_emit<float, float>(i, j, acc[a][b][e], n, k, s, Q, q, diag);
        }
  } else {
    float* dst = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (GB_BM * GB_BM);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int li = wm + a * 16 + out_row + e;
          const int lj = wn + b * 16 + out_col;
          dst[li * GB_BM + lj] = acc[a][b][e];
        }
  }
}

// Sum of split-K partial tiles in fixed split order, then the rescale epilogue.
__global__ __launch_bounds__(256) void gram_splitk_epilogue_kernel(
    int64_t n, int64_t k, const float* __restrict__ partial, int nsplit, int ntiles,
    int tiles_aug, const double* __restrict__ s, float* __restrict__ Q, float* __restrict__ q) {
  int ti, tj;
  decode_tile(blockIdx.x, tiles_aug, ti, tj);
  const bool diag = (ti == tj);
  const int64_t i0 = (int64_t)ti * GB_BM, j0 = (int64_t)tj * GB_BM;
  for (int e = threadIdx.x; e < GB_BM * GB_BM; e += 256) {
    float acc = 0.f;
    for (int sp = 0; sp < nsplit; ++sp)
      acc += partial[((int64_t)sp * ntiles + blockIdx.x) * (GB_BM * GB_BM) + e];
    const int li = e / GB_BM, lj = e % GB_BM;
    gram_emit<float, float>(i0 + li, j0 + lj, acc, n, k, s, Q, q, diag);
  }
}

// ---------------------------------------------------------------------------------------------
// Plain FMA Gram (FP64 or FP32): 64 x 64 tiles, 256 threads with 4 x 4 outputs each.
// ---------------------------------------------------------------------------------------------
constexpr int GF_BM = 64;
constexpr int GF_BK = 16;

template <typename T>
__global__ __launch_bounds__(256) void gram_fma_kernel(int64_t d, int64_t n, int64_t k,
                                                       const T* __restrict__ A, int64_t lda,
                                                       const T* __restrict__ B, int64_t ldb,
                                                       const double* __restrict__ s,
                                                       T* __restrict__ Q, T* __restrict__ q,
                                                       int tiles_aug) {
  __shared__ T sx[GF_BK][GF_BM + 1];
  __shared__ T sy[GF_BK][GF_BM + 1];
  int ti, tj;
  decode_tile(blockIdx.x, tiles_aug, ti, tj);
  const bool diag = (ti == tj);
  const int64_t i0 = (int64_t)ti * GF_BM, j0 = (int64_t)tj * GF_BM;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;

  for (int64_t r0 = 0; r0 < d; r0 += GF_BK) {
    for (int e = threadIdx.x; e < GF_BK * GF_BM; e += 256) {
      const int rr = e / GF_BM, cc = e % GF_BM;
      const int64_t r = r0 + rr;
      T vx = (T)0, vy = (T)0;
      if (r < d) {
        const int64_t cx = i0 + cc, cy = j0 + cc;
        if (cx < n) vx = A[r * lda + cx];
        else if (cx < n + k) vx = B[r * ldb + (cx - n)];
        if (cy < n) vy = A[r * lda + cy];
        else if (cy < n + k) vy = B[r * ldb + (cy - n)];
      }
      sx[rr][cc] = vx;
      sy[rr][cc] = vy;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < GF_BK; ++rr) {
      T xv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = sx[rr][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) yv[b] = sy[rr][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xv[a], yv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      gram_emit<T, T>(i0 + ty + 16 * a, j0 + tx + 16 * b, acc[a][b], n, k, s, Q, q, diag);
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
static int64_t colnorm_chunks(int64_t d, int64_t n) {
  const int64_t bx = (n + 255) / 256;
  int64_t chunks = (2048 + bx - 1) / bx;
  if (chunks > d) chunks = d;
  if (chunks < 1) chunks = 1;
  return chunks;
}

size_t colnorm_ws_bytes(int64_t d, int64_t n) {
  return sizeof(double) * (size_t)(colnorm_chunks(d, n) * n);
}

template <typename T>
hipError_t launch_colnorm(int64_t d, int64_t n, const T* A, int64_t lda, double* s, double* ws,
                          hipStream_t st) {
  const int64_t chunks = colnorm_chunks(d, n);
  const int64_t rows = (d + chunks - 1) / chunks;
  dim3 g1((unsigned)((n + 255) / 256), (unsigned)chunks);
  hipLaunchKernelGGL(colnorm_partial_kernel<T>, g1, dim3(256), 0, st, d, n, A, lda, rows, ws);
  hipLaunchKernelGGL(colnorm_finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     n, chunks, (const double*)ws, s);
  return hipGetLastError();
}
template hipError_t launch_colnorm<float>(int64_t, int64_t, const float*, int64_t, double*,
                                         double*, hipStream_t);
template hipError_t launch_colnorm<double>(int64_t, int64_t, const double*, int64_t, double*,
                                          double*, hipStream_t);

static void gram_tiles(int64_t n, int64_t k, int bm, int& tiles_a, int& tiles_aug, int& ntiles) {
  tiles_a = (int)((n + bm - 1) / bm);
  tiles_aug = (int)((n + k + bm - 1) / bm);
  ntiles = tiles_a * tiles_aug - tiles_a * (tiles_a - 1) / 2;
}

int gram_bf16x3_splits(int64_t d, int64_t n, int64_t k) {
  int ta, taug, nt;
  gram_tiles(n, k, GB_BM, ta, taug, nt);
  int splits = 1;
  // Fewer tiles than about two per compute unit: split the K loop (rows of A).
  while (nt * splits < 512 && d / (splits * 2) >= 4 * GB_BK && splits < 32) splits *= 2;
  return splits;
}

size_t gram_bf16x3_ws_bytes(int64_t d, int64_t n, int64_t k) {
  int ta, taug, nt;
  gram_tiles(n, k, GB_BM, ta, taug, nt);
  const int splits = gram_bf16x3_splits(d, n, k);
  return splits > 1 ? sizeof(float) * (size_t)splits * nt * GB_BM * GB_BM : 0;
}

hipError_t launch_gram_bf16x3(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                              const float* B, int64_t ldb, const double* s, float* Q, float* q,
                              float* ws, hipStream_t st) {
  int ta, taug, nt;
  gram_tiles(n, k, GB_BM, ta, taug, nt);
  const int splits = gram_bf16x3_splits(d, n, k);
  int64_t rows = (d + splits - 1) / splits;
  rows = (rows + GB_BK - 1) / GB_BK * GB_BK;
  dim3 grid((unsigned)nt, (unsigned)splits);
  hipLaunchKernelGGL(gram_bf16x3_kernel, grid, dim3(256), 0, st, d, n, k, A, lda, B, ldb, s, Q, q,
                     splits > 1 ? ws : (float*)nullptr, taug, rows);
  if (splits > 1)
    hipLaunchKernelGGL(gram_splitk_epilogue_kernel, dim3((unsigned)nt), dim3(256), 0, st, n, k,
                       (const float*)ws, splits, nt, taug, s, Q, q);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gram_fma(int64_t d, int64_t n, int64_t k, const T* A, int64_t lda, const T* B,
                           int64_t ldb, const double* s, T* Q, T* q, hipStream_t st) {
  int ta, taug, nt;
  gram_tiles(n, k, GF_BM, ta, taug, nt);
  hipLaunchKernelGGL(gram_fma_kernel<T>, dim3((unsigned)nt), dim3(256), 0, st, d, n, k, A, lda, B,
                     ldb, s, Q, q, taug);
  return hipGetLastError();
}
template hipError_t launch_gram_fma<float>(int64_t, int64_t, int64_t, const float*, int64_t,
                                          const float*, int64_t, const double*, float*, float*,
                                          hipStream_t);
template hipError_t launch_gram_fma<double>(int64_t, int64_t, int64_t, const double*, int64_t,
                                           const double*, int64_t, const double*, double*,
                                           double*, hipStream_t);

}  // namespace nnls
