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
#include <algorithm>

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
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t c = 0;
  for (; c + 3 < nchunks; c += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] += partial[(c + u) * n + col];
  }
  for (; c < nchunks; ++c) a[0] += partial[c * n + col];
  const double acc = (a[0] + a[1]) + (a[2] + a[3]);
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
// 64 x 64), K staged 32 rows at a time through a two-slot LDS ring: while the waves run the
// MFMAs of slot s, the next chunk (already in registers) is converted and written to slot s^1
// and the chunk after it is fetched from memory, so one barrier per K step suffices.
// LDS holds the hi and lo parts of both panels, column-major (32 consecutive k of one column
// contiguous, padded to 40 bf16 = 80 bytes so the 16-byte accesses of 16 consecutive lanes hit
// distinct banks).  The split uses the hardware packed conversion (round to nearest even).
//
// Tile schedule: workgroup b runs on XCD b % 8 (round-robin dispatch).  Tiles are grouped in
// blocks of 4 tile rows x 8 tile columns; group g belongs to XCD g % 8, so the ~32 tiles an XCD
// runs at a time read 4 + 8 panels through its own L2 instead of up to 64.
// ---------------------------------------------------------------------------------------------
constexpr int GB_BM = 128;
constexpr int GB_BK = 32;
constexpr int GB_LDK = 40;  // padded k stride in bf16 units
constexpr int GB_PANEL = GB_BM * GB_LDK;     // bf16 per panel part (hi or lo)
constexpr int GB_SLOT = 4 * GB_PANEL;        // Xh, Xl, Yh, Yl
constexpr int GB_LDS_BYTES = 2 * GB_SLOT * 2;
constexpr int GB_GROUP_ROWS = 4;
constexpr int GB_GROUP_COLS = 8;
constexpr int GB_XCDS = 8;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

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

// Number of tiles (ti, tj), ti <= tj, in group (band, chunk).
__device__ __forceinline__ int group_size(int band, int chunk, int tiles_a, int tiles_aug) {
  const int r0 = band * GB_GROUP_ROWS;
  const int r1 = min(r0 + GB_GROUP_ROWS, tiles_a);
  const int c0 = r0 + chunk * GB_GROUP_COLS;
  const int c1 = min(c0 + GB_GROUP_COLS, tiles_aug);
  int cnt = 0;
  for (int ti = r0; ti < r1; ++ti) {
    const int lo = max(c0, ti);
    cnt += c1 > lo ? c1 - lo : 0;
  }
  return cnt;
}

// Tile of workgroup b under the XCD-grouped schedule; false if b has no tile.
__device__ bool schedule_tile(int b, int tiles_a, int tiles_aug, int& ti, int& tj) {
  const int xcd = b % GB_XCDS;
  int slot = b / GB_XCDS;
  const int bands = (tiles_a + GB_GROUP_ROWS - 1) / GB_GROUP_ROWS;
  int g = 0;
  for (int band = 0; band < bands; ++band) {
    const int r0 = band * GB_GROUP_ROWS;
    const int chunks = (tiles_aug - r0 + GB_GROUP_COLS - 1) / GB_GROUP_COLS;
    for (int chunk = 0; chunk < chunks; ++chunk, ++g) {
      if (g % GB_XCDS != xcd) continue;
      const int sz = group_size(band, chunk, tiles_a, tiles_aug);
      if (slot >= sz) {
        slot -= sz;
        continue;
      }
      const int c0 = r0 + chunk * GB_GROUP_COLS;
      const int c1 = min(c0 + GB_GROUP_COLS, tiles_aug);
      const int r1 = min(r0 + GB_GROUP_ROWS, tiles_a);
      for (int t = r0; t < r1; ++t) {
        const int lo = max(c0, t);
        const int w = c1 > lo ? c1 - lo : 0;
        if (slot < w) {
          ti = t;
          tj = lo + slot;
          return true;
        }
        slot -= w;
      }
    }
  }
  return false;
}

// Host mirror of the schedule: workgroups needed = 8 x the largest per-XCD tile count.
static int schedule_blocks(int tiles_a, int tiles_aug) {
  int per[GB_XCDS] = {0};
  const int bands = (tiles_a + GB_GROUP_ROWS - 1) / GB_GROUP_ROWS;
  int g = 0;
  for (int band = 0; band < bands; ++band) {
    const int r0 = band * GB_GROUP_ROWS;
    const int chunks = (tiles_aug - r0 + GB_GROUP_COLS - 1) / GB_GROUP_COLS;
    for (int chunk = 0; chunk < chunks; ++chunk, ++g) {
      const int c0 = r0 + chunk * GB_GROUP_COLS;
      const int c1 = std::min(c0 + GB_GROUP_COLS, tiles_aug);
      const int r1 = std::min(r0 + GB_GROUP_ROWS, tiles_a);
      int cnt = 0;
      for (int ti = r0; ti < r1; ++ti) {
        const int lo = std::max(c0, ti);
        cnt += c1 > lo ? c1 - lo : 0;
      }
      per[g % GB_XCDS] += cnt;
    }
  }
  int mx = 0;
  for (int x = 0; x < GB_XCDS; ++x) mx = std::max(mx, per[x]);
  return mx * GB_XCDS;
}

// One 128 x 128 tile of [A | B]^T [A | B] over rows [r_begin, r_end): px / py locate the two
// panels (this thread's column of each), diag marks px == py.  Leaves the FP32 accumulators in
// acc (16x16 MFMA D layout) and LDS free for reuse.  Called by all 256 threads.
__device__ __forceinline__ void gram_tile_bf16x3(f32x4 (&acc)[4][4], int64_t r_begin,
                                                 int64_t r_end, GramPanelPtr px, GramPanelPtr py,
                                                 bool diag, uint16_t* lds) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lc = tid & 127;     // column of the panel this thread stages
  const int kh = tid >> 7;      // which 16-row half of the K chunk

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
  // hi / lo split of one pair of staged values (hardware round to nearest even)
  auto split_pair = [](float v0, float v1, uint32_t& h, uint32_t& l) {
    const f32x2 x = {v0, v1};
    const bf16x2 hb = __builtin_convertvector(x, bf16x2);
    const f32x2 hf = __builtin_convertvector(hb, f32x2);
    const bf16x2 lb = __builtin_convertvector(x - hf, bf16x2);
    h = __builtin_bit_cast(uint32_t, hb);
    l = __builtin_bit_cast(uint32_t, lb);
  };
  uint32_t hx[8], lx[8], hy[8], ly[8];
  auto write_chunk = [&](int slot) {
    uint16_t* base = lds + slot * GB_SLOT;
    const int off = lc * GB_LDK + kh * 16;
    *(u32x4*)&base[off] = (u32x4){hx[0], hx[1], hx[2], hx[3]};
    *(u32x4*)&base[off + 8] = (u32x4){hx[4], hx[5], hx[6], hx[7]};
    *(u32x4*)&base[GB_PANEL + off] = (u32x4){lx[0], lx[1], lx[2], lx[3]};
    *(u32x4*)&base[GB_PANEL + off + 8] = (u32x4){lx[4], lx[5], lx[6], lx[7]};
    if (!diag) {
      *(u32x4*)&base[2 * GB_PANEL + off] = (u32x4){hy[0], hy[1], hy[2], hy[3]};
      *(u32x4*)&base[2 * GB_PANEL + off + 8] = (u32x4){hy[4], hy[5], hy[6], hy[7]};
      *(u32x4*)&base[3 * GB_PANEL + off] = (u32x4){ly[0], ly[1], ly[2], ly[3]};
      *(u32x4*)&base[3 * GB_PANEL + off + 8] = (u32x4){ly[4], ly[5], ly[6], ly[7]};
    }
  };

  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  const int frag_row = lane & 15;
  const int frag_k = (lane >> 4) * 8;

  const int64_t nsteps = r_end > r_begin ? (r_end - r_begin + GB_BK - 1) / GB_BK : 0;
  if (nsteps > 0) {
    load_chunk(r_begin);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      split_pair(rx[2 * u], rx[2 * u + 1], hx[u], lx[u]);
      split_pair(ry[2 * u], ry[2 * u + 1], hy[u], ly[u]);
    }
    write_chunk(0);
    if (nsteps > 1) load_chunk(r_begin + GB_BK);
    __syncthreads();
  }
  for (int64_t step = 0; step < nsteps; ++step) {
    const int slot = (int)(step & 1);
    const uint16_t* xh = lds + slot * GB_SLOT;
    const uint16_t* xl = xh + GB_PANEL;
    const uint16_t* yh = diag ? xh : xh + 2 * GB_PANEL;
    const uint16_t* yl = diag ? xl : xh + 3 * GB_PANEL;
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int xo = (wm + t * 16 + frag_row) * GB_LDK + frag_k;
      const int yo = (wn + t * 16 + frag_row) * GB_LDK + frag_k;
      ah[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&xh[xo]);
      al[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&xl[xo]);
      bh[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&yh[yo]);
      bl[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&yl[yo]);
    }
    // MFMAs of this slot with the split of the staged next chunk interleaved: the conversion
    // is independent register work the wave issues while the matrix core is busy.  (On the
    // last step the staged registers hold stale values; converting and writing them to the
    // idle slot is harmless.)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int u = 2 * a; u < 2 * a + 2; ++u) {
        split_pair(rx[2 * u], rx[2 * u + 1], hx[u], lx[u]);
        split_pair(ry[2 * u], ry[2 * u + 1], hy[u], ly[u]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
      }
      // the staged registers are free once the last pair is split
      if (a == 3 && step + 2 < nsteps) load_chunk(r_begin + (step + 2) * GB_BK);
    }
    write_chunk(slot ^ 1);
    __syncthreads();
  }

}

__global__ __launch_bounds__(256, 2) void gram_bf16x3_kernel(
    int64_t d, int64_t n, int64_t k, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, const double* __restrict__ s, float* __restrict__ Q,
    float* __restrict__ q, float* __restrict__ partial, int tiles_a, int tiles_aug,
    int64_t rows_per_split) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];

  int ti, tj;
  if (!schedule_tile(blockIdx.x, tiles_a, tiles_aug, ti, tj)) return;
  const bool diag = (ti == tj);
  const int64_t i0 = (int64_t)ti * GB_BM, j0 = (int64_t)tj * GB_BM;
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r_end = r_begin + rows_per_split < d ? r_begin + rows_per_split : d;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lc = tid & 127;
  const GramPanelPtr px = panel_column(i0 + lc, n, k, A, lda, B, ldb);
  const GramPanelPtr py = panel_column(j0 + lc, n, k, A, lda, B, ldb);
  f32x4 acc[4][4];
  gram_tile_bf16x3(acc, r_begin, r_end, px, py, diag, lds);
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;

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
    // partial tiles are indexed by (ti, tj) in the plain row-major tile order
    int tile = 0;
    for (int t = 0; t < ti; ++t) tile += tiles_aug - t;
    tile += tj - ti;
    const int ntiles = tiles_a * tiles_aug - tiles_a * (tiles_a - 1) / 2;
    float* dst = partial + ((int64_t)blockIdx.y * ntiles + tile) * (GB_BM * GB_BM);
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

// ---------------------------------------------------------------------------------------------
// Uneven batch: one workgroup per problem walks that problem's tiles of [A | b]^T [A | b] with
// the same BF16x3 tile routine.  Diagonal tiles go first; each yields the scales of its block
// from its own diagonal (s_i = sqrt(H_ii), 1 where H_ii = 0), which the off-diagonal tiles and
// the right-hand side column then use in the rescale epilogue.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void batched_emit(int64_t i, int64_t j, float val, int64_t n,
                                             const double* s_l, float* Q, float* q,
                                             bool diag_tile) {
  if (i >= n) return;
  if (j < n) {
    if (diag_tile && i > j) return;
    float out;
    if (i == j) out = val > 0.f ? 1.f : 0.f;
    else out = (float)((double)val / (s_l[i] * s_l[j]));
    Q[i * n + j] = out;
    if (i != j) Q[j * n + i] = out;
  } else if (j == n) {
    q[i] = (float)(-(double)val / s_l[i]);
  }
}

constexpr int BG_MAX_N = 1024;

__global__ __launch_bounds__(256, 1) void batched_gram_kernel(const BatchDesc* __restrict__ desc,
                                                           const float* __restrict__ A_pool,
                                                           const float* __restrict__ B_pool,
                                                           float* __restrict__ Q_pool,
                                                           float* __restrict__ q_pool,
                                                           double* __restrict__ s_pool) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  double* s_l = (double*)((unsigned char*)lds + GB_LDS_BYTES);
  float* dg = (float*)(s_l + BG_MAX_N);
  const BatchDesc D = desc[blockIdx.x];
  const int64_t n = D.n, d = D.d;
  const float* A = A_pool + D.offA;
  const float* B = B_pool + D.offB;
  float* Q = Q_pool + D.offQ;
  float* q = q_pool + D.offq;
  const int T = (int)((n + GB_BM - 1) / GB_BM);
  const int Taug = (int)((n + 1 + GB_BM - 1) / GB_BM);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lc = tid & 127;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int out_col = lane & 15, out_row = (lane >> 4) * 4;
  f32x4 acc[4][4];
  for (int pass = 0; pass < 2; ++pass) {
    for (int ti = 0; ti < T; ++ti) {
      const int tj_lo = pass == 0 ? ti : ti + 1;
      const int tj_hi = pass == 0 ? ti + 1 : Taug;
      for (int tj = tj_lo; tj < tj_hi; ++tj) {
        const bool diag = ti == tj;
        const int64_t i0 = (int64_t)ti * GB_BM, j0 = (int64_t)tj * GB_BM;
        const GramPanelPtr px = panel_column(i0 + lc, n, 1, A, n, B, 1);
        const GramPanelPtr py = panel_column(j0 + lc, n, 1, A, n, B, 1);
        gram_tile_bf16x3(acc, 0, d, px, py, diag, lds);
        if (diag) {
          // diagonal entries of the block -> scales
          if (wm == wn) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int e = out_col - out_row;
              if (e >= 0 && e < 4) {
#pragma unroll
                for (int ee = 0; ee < 4; ++ee)
                  if (ee == e) dg[wm + a * 16 + out_col] = acc[a][a][ee];
              }
            }
          }
          __syncthreads();
          if (tid < GB_BM) {
            const int64_t i = i0 + tid;
            if (i < n) {
              const float h = dg[tid];
              const double si = h > 0.f ? sqrt((double)h) : 1.0;
              s_l[i] = si;
              s_pool[D.offq + i] = si;
            }
          }
          __syncthreads();
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              batched_emit(i0 + wm + a * 16 + out_row + e, j0 + wn + b * 16 + out_col,
                           acc[a][b][e], n, s_l, Q, q, diag);
      }
    }
  }
}

size_t batched_gram_lds_bytes() {
  return GB_LDS_BYTES + sizeof(double) * BG_MAX_N + sizeof(float) * GB_BM;
}

hipError_t prepare_batched_gram() {
  return hipFuncSetAttribute((const void*)batched_gram_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)batched_gram_lds_bytes());
}

hipError_t launch_batched_gram(const BatchDesc* desc, int64_t count, const float* A_pool,
                               const float* B_pool, float* Q_pool, float* q_pool,
                               double* s_pool, hipStream_t st) {
  const size_t lds = batched_gram_lds_bytes();
  hipLaunchKernelGGL(batched_gram_kernel, dim3((unsigned)count), dim3(256), lds, st, desc, A_pool,
                     B_pool, Q_pool, q_pool, s_pool);
  return hipGetLastError();
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
  if (chunks > 256) chunks = 256;  // the finalize pass sums this many partials per column
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
  const int blocks = schedule_blocks(ta, taug);
  dim3 grid((unsigned)blocks, (unsigned)splits);
  hipError_t e = hipFuncSetAttribute((const void*)gram_bf16x3_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, GB_LDS_BYTES);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_bf16x3_kernel, grid, dim3(256), GB_LDS_BYTES, st, d, n, k, A, lda, B,
                     ldb, s, Q, q, splits > 1 ? ws : (float*)nullptr, ta, taug, rows);
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
