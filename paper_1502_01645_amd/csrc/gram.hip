// Gram product and rescale of Algorithm 1 (Problem (2) -> Problem (5)) for gfx950.
//
//   colnorm     s_i = ||A_i||_2 in FP64 from the stored entries (1 for a zero column)
//   presplit +  upper-triangle tiles of [A | B]^T [A | B] restricted to rows of A, so one launch
//   gram_dma    gives H = A^T A and A^T B.  FP32 inputs are split once into hi + lo bfloat16
//               (presplit, stored by column); each 256 x 256 tile streams both parts through
//               LDS with direct global-to-LDS loads and accumulates hi*hi + hi*lo + lo*hi on the
//               matrix cores (v_mfma_f32_16x16x32_bf16) in FP32.  The epilogue applies the
//               rescale of Problem (5) directly: Q_ij = H_ij / (s_i s_j), Q_ii = 1,
//               q = -A^T B / s, and mirrors the tile into the lower triangle.  Split-K over the
//               rows of A fills the GPU when there are few tiles; the partial tiles then go
//               through gram_splitk_epilogue.
//   batched     the tiles of an uneven batch of problems as independent work items, 64 x 64 or
//               128 x 128 by size class, split while they are staged (gram_tile_bf16x3).
//   gram_fma    the same product with plain FMAs in FP32 or FP64 (FP64 problems and the FP32
//               accuracy cross-check).
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

// Block: 16 columns; thread (column tid % 16, group tid / 16) sums the chunks g, g + 16, ... with
// four accumulators, then the 16 group sums of a column are added in fixed order.  (A wave reads
// 16 consecutive doubles of 4 chunks at a time; 16 columns per block give enough blocks to
// spread the partial sums over the GPU.)
constexpr int CN_C = 16;
constexpr int CN_G = 256 / CN_C;
__global__ __launch_bounds__(256) void colnorm_finalize_kernel(int64_t n, int64_t nchunks,
                                                               const double* partial, double* s) {
  __shared__ double red[CN_G][CN_C];
  const int cl = threadIdx.x % CN_C, grp = threadIdx.x / CN_C;
  const int64_t col = (int64_t)blockIdx.x * CN_C + cl;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (col < n) {
    int64_t c = grp;
    for (; c + 3 * CN_G < nchunks; c += 4 * CN_G) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += partial[(c + CN_G * u) * n + col];
    }
    for (; c < nchunks; c += CN_G) a[0] += partial[c * n + col];
  }
  red[grp][cl] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  if (grp == 0 && col < n) {
    double acc = 0.0;
#pragma unroll
    for (int g = 0; g < CN_G; ++g) acc += red[g][cl];
    s[col] = acc > 0.0 ? sqrt(acc) : 1.0;
  }
}

// ---------------------------------------------------------------------------------------------
// Epilogue shared by all Gram variants: one entry (i, j) of [A | B]^T [A | B] with i < n.
// ---------------------------------------------------------------------------------------------
// Q is written from one computed value per unordered pair {i, j}, so it is exactly symmetric:
// tiles above the diagonal mirror every entry; in diagonal tiles only i <= j is emitted.  With
// s == nullptr nothing is rescaled: Q = H (its diagonal included) and q = -A^T B.
template <typename T, typename Acc>
__device__ __forceinline__ void gram_emit(int64_t i, int64_t j, Acc val, int64_t n, int64_t k,
                                          const double* __restrict__ s, T* __restrict__ Q,
                                          T* __restrict__ q, bool diag_tile) {
  if (i >= n) return;
  if (j < n) {
    if (diag_tile && i > j) return;
    T out;
    if (s == nullptr) {
      out = (T)val;
    } else if (i == j) {
      out = val > (Acc)0 ? (T)1 : (T)0;
    } else {
      out = (T)((double)val / (s[i] * s[j]));
    }
    Q[i * n + j] = out;
    if (i != j) Q[j * n + i] = out;
  } else if (j < n + k) {
    q[i * k + (j - n)] = s == nullptr ? (T)(-val) : (T)(-(double)val / s[i]);
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
// BF16x3 Gram on the matrix cores for the uneven batch: a BM x BM tile (BM = 64 or 128) per
// workgroup of 4 waves (2 x 2 waves of BM/2 x BM/2), K staged 32 rows at a time through a
// two-slot LDS ring: while the waves run the MFMAs of slot s, the next chunk (already in
// registers) is converted and written to slot s^1 and the chunk after it is fetched from
// memory, so one barrier per K step suffices.  LDS holds the hi and lo parts of both panels,
// column-major (32 consecutive k of one column contiguous, padded to 40 bf16 = 80 bytes so the
// 16-byte accesses of 16 consecutive lanes hit distinct banks).  The split uses the hardware
// packed conversion (round to nearest even).
//
// The single-problem schedule (gram_dma below) deals its tiles to XCDs in groups of 4 tile rows
// x 8 tile columns, so the ~32 tiles an XCD runs at a time read 4 + 8 panels through its own L2
// instead of up to 64.
// ---------------------------------------------------------------------------------------------
constexpr int GB_BK = 32;
constexpr int GB_LDK = 40;  // padded k stride in bf16 units

template <int BM>
struct GbTile {
  static constexpr int MT = BM / 32;        // 16 x 16 blocks per wave in each direction
  static constexpr int TPC = 256 / BM;      // threads staging one panel column
  static constexpr int RPT = GB_BK / TPC;   // rows of a K chunk one staging thread loads
  static constexpr int PANEL = BM * GB_LDK; // bf16 per panel part (hi or lo)
  static constexpr int SLOT = 4 * PANEL;    // Xh, Xl, Yh, Yl
  static constexpr int LDS_BYTES = 2 * SLOT * 2;
  static_assert(BM == 64 || BM == 128, "tile size");
  static_assert(RPT % 8 == 0 && RPT / 2 == 2 * MT, "staging split interleave");
};
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
__host__ __device__ inline int group_size(int band, int chunk, int tiles_a, int tiles_aug) {
  const int r0 = band * GB_GROUP_ROWS;
  const int r1 = r0 + GB_GROUP_ROWS < tiles_a ? r0 + GB_GROUP_ROWS : tiles_a;
  const int c0 = r0 + chunk * GB_GROUP_COLS;
  const int c1 = c0 + GB_GROUP_COLS < tiles_aug ? c0 + GB_GROUP_COLS : tiles_aug;
  int cnt = 0;
  for (int ti = r0; ti < r1; ++ti) {
    const int lo = c0 > ti ? c0 : ti;
    cnt += c1 > lo ? c1 - lo : 0;
  }
  return cnt;
}

// Tile t of the grouped order: groups of 4 tile rows x 8 tile columns (band by band, chunk by
// chunk), row-major inside a group, so neighbours in the order share panels.
__device__ void grouped_tile(int t, int tiles_a, int tiles_aug, int& ti, int& tj) {
  const int bands = (tiles_a + GB_GROUP_ROWS - 1) / GB_GROUP_ROWS;
  for (int band = 0; band < bands; ++band) {
    const int r0 = band * GB_GROUP_ROWS;
    const int chunks = (tiles_aug - r0 + GB_GROUP_COLS - 1) / GB_GROUP_COLS;
    for (int chunk = 0; chunk < chunks; ++chunk) {
      const int sz = group_size(band, chunk, tiles_a, tiles_aug);
      if (t >= sz) {
        t -= sz;
        continue;
      }
      const int c0 = r0 + chunk * GB_GROUP_COLS;
      const int c1 = min(c0 + GB_GROUP_COLS, tiles_aug);
      const int r1 = min(r0 + GB_GROUP_ROWS, tiles_a);
      for (int r = r0; r < r1; ++r) {
        const int lo = max(c0, r);
        const int w = c1 > lo ? c1 - lo : 0;
        if (t < w) {
          ti = r;
          tj = lo + t;
          return;
        }
        t -= w;
      }
    }
  }
  ti = tj = 0;  // not reached for t < ntiles
}

// Work item of workgroup b: items are (split, tile) pairs, split-major over the grouped tile
// order.  Workgroup b runs on XCD b % 8 (round-robin dispatch); XCD x takes the x-th contiguous
// eighth of the item list, so each XCD holds a balanced share of neighbouring tiles and the
// panels they share stay in its own L2.  False if b has no item.
__device__ bool schedule_item(int b, int ntiles, int splits, int tiles_a, int tiles_aug, int& ti,
                              int& tj, int& split) {
  const int items = ntiles * splits;
  const int per = (items + GB_XCDS - 1) / GB_XCDS;
  const int slot = b / GB_XCDS;
  if (slot >= per) return false;
  const int idx = (b % GB_XCDS) * per + slot;
  if (idx >= items) return false;
  split = idx / ntiles;
  grouped_tile(idx % ntiles, tiles_a, tiles_aug, ti, tj);
  return true;
}

static int schedule_blocks(int ntiles, int splits) {
  const int items = ntiles * splits;
  return (items + GB_XCDS - 1) / GB_XCDS * GB_XCDS;
}

// One BM x BM tile of [A | B]^T [A | B] over rows [r_begin, r_end): px / py locate the two
// panels (this thread's column of each), diag marks px == py.  Leaves the FP32 accumulators in
// acc (16x16 MFMA D layout) and LDS free for reuse.  Called by all 256 threads.
template <int BM>
__device__ __forceinline__ void gram_tile_bf16x3(f32x4 (&acc)[BM / 32][BM / 32],
                                                 int64_t r_begin, int64_t r_end, GramPanelPtr px,
                                                 GramPanelPtr py, bool diag, uint16_t* lds) {
  using G = GbTile<BM>;
  constexpr int MT = G::MT, RPT = G::RPT, NP = RPT / 2;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lc = tid % BM;      // column of the panel this thread stages
  const int kh = tid / BM;      // which RPT-row part of the K chunk

#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

  float rx[RPT], ry[RPT];
  auto load_chunk = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int64_t r = r0 + kh * RPT + u;
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
  uint32_t hx[NP], lx[NP], hy[NP], ly[NP];
  auto write_chunk = [&](int slot) {
    uint16_t* base = lds + slot * G::SLOT;
    const int off = lc * GB_LDK + kh * RPT;
#pragma unroll
    for (int v = 0; v < NP / 4; ++v) {
      const int o = off + 8 * v;
      *(u32x4*)&base[o] = (u32x4){hx[4 * v], hx[4 * v + 1], hx[4 * v + 2], hx[4 * v + 3]};
      *(u32x4*)&base[G::PANEL + o] =
          (u32x4){lx[4 * v], lx[4 * v + 1], lx[4 * v + 2], lx[4 * v + 3]};
      if (!diag) {
        *(u32x4*)&base[2 * G::PANEL + o] =
            (u32x4){hy[4 * v], hy[4 * v + 1], hy[4 * v + 2], hy[4 * v + 3]};
        *(u32x4*)&base[3 * G::PANEL + o] =
            (u32x4){ly[4 * v], ly[4 * v + 1], ly[4 * v + 2], ly[4 * v + 3]};
      }
    }
  };

  const int wm = (wave >> 1) * (BM / 2);
  const int wn = (wave & 1) * (BM / 2);
  const int frag_row = lane & 15;
  const int frag_k = (lane >> 4) * 8;

  const int64_t nsteps = r_end > r_begin ? (r_end - r_begin + GB_BK - 1) / GB_BK : 0;
  if (nsteps > 0) {
    load_chunk(r_begin);
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      split_pair(rx[2 * u], rx[2 * u + 1], hx[u], lx[u]);
      split_pair(ry[2 * u], ry[2 * u + 1], hy[u], ly[u]);
    }
    write_chunk(0);
    if (nsteps > 1) load_chunk(r_begin + GB_BK);
    __syncthreads();
  }
  for (int64_t step = 0; step < nsteps; ++step) {
    const int slot = (int)(step & 1);
    const uint16_t* xh = lds + slot * G::SLOT;
    const uint16_t* xl = xh + G::PANEL;
    const uint16_t* yh = diag ? xh : xh + 2 * G::PANEL;
    const uint16_t* yl = diag ? xl : xh + 3 * G::PANEL;
    bf16x8 ah[MT], al[MT], bh[MT], bl[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
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
    for (int a = 0; a < MT; ++a) {
#pragma unroll
      for (int u = 2 * a; u < 2 * a + 2; ++u) {
        split_pair(rx[2 * u], rx[2 * u + 1], hx[u], lx[u]);
        split_pair(ry[2 * u], ry[2 * u + 1], hy[u], ly[u]);
      }
#pragma unroll
      for (int b = 0; b < MT; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
      }
      // the staged registers are free once the last pair is split
      if (a == MT - 1 && step + 2 < nsteps) load_chunk(r_begin + (step + 2) * GB_BK);
    }
    write_chunk(slot ^ 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// BF16x3 Gram with pre-split operands and direct-to-LDS loads (the single-problem path).
//
// presplit_kernel writes [A | B] once as two BF16 matrices (hi and lo of the split), stored by
// column: column c is dpad consecutive values (zero past d, zero columns up to the padded width),
// so the K direction of the Gram is contiguous and the main loop needs no bounds checks.
//
// gram_dma_kernel: 256 x 256 output tile per workgroup of 8 waves (2 x 4 waves of 128 x 64), K
// staged 32 rows at a time in two LDS stages of 64 KB (Xh, Xl, Yh, Yl parts of 256 columns x 32
// values).  Each stage is filled by global_load_lds_dwordx4 (16 bytes per lane straight into
// LDS): the loads of step s+1 are issued right after the barrier of step s and land while the
// waves run the 3 x 32 MFMAs (hi*hi + hi*lo + lo*hi, v_mfma_f32_16x16x32_bf16) of step s; the
// LDS reads of the next 16-row A fragment pair are placed under the MFMAs of the current one
// (scheduling group barriers), so they do not stall the matrix cores.
// Inside a stage, the four 16-byte k-groups of a column are stored XOR-swizzled by gd_swz of the
// column, so the fragment reads of 8 or 16 consecutive columns hit distinct bank groups.  The
// swizzle is applied on the global side: lane i of a load instruction fetches the k-group that
// belongs at LDS position i.  One barrier per step: waits are explicit (vmcnt for this wave's
// own loads of the step, lgkmcnt for its last LDS reads) and the barrier is a bare s_barrier,
// so the loads of the next step stay in flight across it.
// ---------------------------------------------------------------------------------------------
constexpr int PS_T = 64;
constexpr int GD_T = 256;
constexpr int GD_BK = 32;
constexpr int GD_WAVES_N = 4;               // waves across the tile's columns (2 across rows)
constexpr int GD_NT = 2 * GD_WAVES_N * 64;
constexpr int GD_PART = GD_T * GD_BK;        // bf16 per part
constexpr int GD_STAGE = 4 * GD_PART;
constexpr int GD_LDS_BYTES = 2 * GD_STAGE * 2;
constexpr int GD_CPI = 512 / GD_BK;          // columns per load instruction (1 KB)
constexpr int GD_IPP = GD_T / GD_CPI;        // instructions per part
constexpr int GD_IPW = 4 * GD_IPP / (GD_NT / 64);
constexpr int GD_MT = 8, GD_NTL = 16 / GD_WAVES_N;  // 16 x 16 blocks per wave (rows, columns)

// LDS position of k-group g of column c (64 bytes per column, four 16-byte k-groups): g ^ swz(c).
// Any 8 consecutive columns (and any 16) then put their 16-byte pieces on distinct bank groups
// whether a fragment read serves 8 lanes per cycle over 128 bytes of banks or 16 lanes over 256.
__device__ __forceinline__ int gd_swz(int c) { return ((c >> 1) ^ (c >> 2)) & 3; }

typedef __attribute__((address_space(1))) void gd_gvoid;
typedef __attribute__((address_space(3))) void gd_lvoid;

__device__ __forceinline__ void gb_split_pair(float v0, float v1, uint32_t& h, uint32_t& l) {
  const f32x2 x = {v0, v1};
  const bf16x2 hb = __builtin_convertvector(x, bf16x2);
  const f32x2 hf = __builtin_convertvector(hb, f32x2);
  const bf16x2 lb = __builtin_convertvector(x - hf, bf16x2);
  h = __builtin_bit_cast(uint32_t, hb);
  l = __builtin_bit_cast(uint32_t, lb);
}

// Grid (ncols_pad / 64, dpad / 64): a 64 x 64 block through LDS, transposed on the way out.
// With colsq != nullptr the block also writes, for its columns of A, the FP64 sum of squares of
// its 64 rows: colsq[row block][column], the partial sums of the column norms.
__global__ __launch_bounds__(256) void presplit_kernel(int64_t d, int64_t n, int64_t k,
                                                       const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ B, int64_t ldb,
                                                       int64_t dpad, uint16_t* __restrict__ Ph,
                                                       uint16_t* __restrict__ Pl,
                                                       double* __restrict__ colsq) {
  __shared__ float t[PS_T][PS_T + 1];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * PS_T, r0 = (int64_t)blockIdx.y * PS_T;
  // a block inside A (or inside B) with 16-byte aligned rows loads 4 columns per lane
  const float* vbase = nullptr;
  int64_t vld = 0;
  if (c0 + PS_T <= n) {
    vbase = A + c0;
    vld = lda;
  } else if (c0 >= n && c0 + PS_T <= n + k) {
    vbase = B + (c0 - n);
    vld = ldb;
  }
  if (vbase != nullptr && ((vld & 3) != 0 || (((uintptr_t)vbase) & 15) != 0)) vbase = nullptr;
  if (vbase != nullptr) {
    const int cq = tid & 15;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = (tid >> 4) + 16 * u;
      const int64_t r = r0 + rr;
      f32x4 v = (f32x4){0.f, 0.f, 0.f, 0.f};
      if (r < d) v = *(const f32x4*)(vbase + r * vld + 4 * cq);
      t[rr][4 * cq + 0] = v[0];
      t[rr][4 * cq + 1] = v[1];
      t[rr][4 * cq + 2] = v[2];
      t[rr][4 * cq + 3] = v[3];
    }
  } else {
    const int tc = tid & (PS_T - 1);
    const int64_t c = c0 + tc;
    const float* colp = nullptr;
    int64_t ld = 0;
    if (c < n) {
      colp = A + c;
      ld = lda;
    } else if (c < n + k) {
      colp = B + (c - n);
      ld = ldb;
    }
    for (int rr = tid >> 6; rr < PS_T; rr += 4) {
      const int64_t r = r0 + rr;
      t[rr][tc] = (colp != nullptr && r < d) ? colp[r * ld] : 0.f;
    }
  }
  __syncthreads();
  // 8 lanes per column, each 8 consecutive rows: every group of 8 lanes writes 128 contiguous
  // bytes of Ph and of Pl
  const int oct = tid & 7;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int cl = pass * 32 + (tid >> 3);
    uint32_t h[4], l[4];
    double sq = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float v0 = t[oct * 8 + 2 * u][cl], v1 = t[oct * 8 + 2 * u + 1][cl];
      gb_split_pair(v0, v1, h[u], l[u]);
      sq += (double)v0 * (double)v0 + (double)v1 * (double)v1;
    }
    const int64_t o = (c0 + cl) * dpad + r0 + oct * 8;
    *(u32x4*)(Ph + o) = (u32x4){h[0], h[1], h[2], h[3]};
    *(u32x4*)(Pl + o) = (u32x4){l[0], l[1], l[2], l[3]};
    if (colsq != nullptr) {
      // the 8 lanes of a column are consecutive: sum over them in fixed order
      sq += __shfl_xor(sq, 1, 64);
      sq += __shfl_xor(sq, 2, 64);
      sq += __shfl_xor(sq, 4, 64);
      if (oct == 0 && c0 + cl < n) colsq[(int64_t)blockIdx.y * n + c0 + cl] = sq;
    }
  }
}

__global__ __launch_bounds__(GD_NT, 1) void gram_dma_kernel(
    int64_t n, int64_t k, const uint16_t* __restrict__ Ph, const uint16_t* __restrict__ Pl,
    int64_t dpad, const double* __restrict__ s, float* __restrict__ Q, float* __restrict__ q,
    float* __restrict__ partial, int tiles_a, int tiles_aug, int ntiles, int nsplit,
    int64_t rows_per_split) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  int ti, tj, split;
  if (!schedule_item(blockIdx.x, ntiles, nsplit, tiles_a, tiles_aug, ti, tj, split)) return;
  const bool diag = (ti == tj);
  const int64_t i0 = (int64_t)ti * GD_T, j0 = (int64_t)tj * GD_T;
  const int64_t r_begin = (int64_t)split * rows_per_split;
  const int64_t r_end = r_begin + rows_per_split < dpad ? r_begin + rows_per_split : dpad;
  const int nsteps = r_end > r_begin ? (int)((r_end - r_begin) / GD_BK) : 0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // this lane's part of each load instruction: column (lane / 4) of the instruction's 16, the
  // k-group that belongs at LDS position lane % 4
  const int lcol = lane >> 2;
  const int lg = (lane & 3) ^ gd_swz(lcol);
  auto issue = [&](int step, int stage) {
#pragma unroll
    for (int u = 0; u < GD_IPW; ++u) {
      const int inst = wave * GD_IPW + u;
      const int part = inst / GD_IPP;
      const int icol0 = (inst % GD_IPP) * GD_CPI;
      const uint16_t* base = (part & 1) ? Pl : Ph;
      const int64_t gc = ((part < 2) ? i0 : j0) + icol0 + lcol;
      const uint16_t* src = base + gc * dpad + r_begin + (int64_t)step * GD_BK + 8 * lg;
      uint16_t* dst = lds + stage * GD_STAGE + part * GD_PART + icol0 * GD_BK;
      __builtin_amdgcn_global_load_lds((gd_gvoid*)src, (gd_lvoid*)dst, 16, 0, 0);
    }
  };

  f32x4 acc[GD_MT][GD_NTL];
#pragma unroll
  for (int a = 0; a < GD_MT; ++a)
#pragma unroll
    for (int b = 0; b < GD_NTL; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int wm = (wave / GD_WAVES_N) * 128, wn = (wave % GD_WAVES_N) * (GD_T / GD_WAVES_N);
  const int fr = lane & 15;
  const int fp = (lane >> 4) ^ gd_swz(fr);  // physical k-group of this lane's fragment

  if (nsteps > 0) issue(0, 0);
  for (int step = 0; step < nsteps; ++step) {
    // own loads of this step done (vmcnt 0), own LDS reads of the previous step done
    // (lgkmcnt 0), then the bare barrier: every wave's part of the stage has landed and the
    // other stage is free for the next step's loads.
    __builtin_amdgcn_s_waitcnt(0x0070);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (step + 1 < nsteps) issue(step + 1, (step + 1) & 1);
    const uint16_t* st = lds + (step & 1) * GD_STAGE;
    bf16x8 bh[GD_NTL], bl[GD_NTL];
#pragma unroll
    for (int t = 0; t < GD_NTL; ++t) {
      const int yo = (wn + t * 16 + fr) * GD_BK + 8 * fp;
      bh[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&st[2 * GD_PART + yo]);
      bl[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&st[3 * GD_PART + yo]);
    }
    // the A fragments of row block a + 1 are read while the MFMAs of block a run
    const int xo0 = (wm + fr) * GD_BK + 8 * fp;
    bf16x8 ahn = __builtin_bit_cast(bf16x8, *(const u32x4*)&st[xo0]);
    bf16x8 aln = __builtin_bit_cast(bf16x8, *(const u32x4*)&st[GD_PART + xo0]);
#pragma unroll
    for (int a = 0; a < GD_MT; ++a) {
      const bf16x8 ah = ahn, al = aln;
      if (a + 1 < GD_MT) {
        const int xo = xo0 + (a + 1) * 16 * GD_BK;
        ahn = __builtin_bit_cast(bf16x8, *(const u32x4*)&st[xo]);
        aln = __builtin_bit_cast(bf16x8, *(const u32x4*)&st[GD_PART + xo]);
      }
#pragma unroll
      for (int b = 0; b < GD_NTL; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[b], acc[a][b], 0, 0, 0);
      }
    }
    // instruction order of the step: the B fragments and the first A pair, then per row block
    // 2 MFMAs, the LDS reads of the next A pair, and the block's other 10 MFMAs, so each read
    // has a block of MFMAs to land under
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * GD_NTL + 2, 0);
#pragma unroll
    for (int a = 0; a + 1 < GD_MT; ++a) {
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * GD_NTL - 2, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 3 * GD_NTL, 0);
  }

  // D fragment layout of the 16x16 FP32 MFMA: lane holds column (lane & 15), rows
  // 4 (lane >> 4) + e.
  const int out_col = lane & 15;
  const int out_row = (lane >> 4) * 4;
  if (partial == nullptr) {
#pragma unroll
    for (int a = 0; a < GD_MT; ++a)
#pragma unroll
      for (int b = 0; b < GD_NTL; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t i = i0 + wm + a * 16 + out_row + e;
          const int64_t j = j0 + wn + b * 16 + out_col;
          gram_emit<float, float>(i, j, acc[a][b][e], n, k, s, Q, q, diag);
        }
  } else {
    int tile = 0;
    for (int t = 0; t < ti; ++t) tile += tiles_aug - t;
    tile += tj - ti;
    float* dst = partial + ((int64_t)split * ntiles + tile) * (GD_T * GD_T);
#pragma unroll
    for (int a = 0; a < GD_MT; ++a)
#pragma unroll
      for (int b = 0; b < GD_NTL; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int li = wm + a * 16 + out_row + e;
          const int lj = wn + b * 16 + out_col;
          dst[li * GD_T + lj] = acc[a][b][e];
        }
  }
}

// ---------------------------------------------------------------------------------------------
// Uneven batch.  The work items are tiles (problem p, ti, tj) of p's [A | b]^T [A | b] at the
// tile size BM of p's size class, in two launches: the diagonal tiles first, each of which
// yields the scales of its block from its own computed diagonal (s_i = sqrt(H_ii), 1 where
// H_ii = 0) and emits its upper triangle rescaled; then the tiles above the diagonal (and the
// right-hand-side column), which read the scales of both blocks back from s_pool.  Every tile is
// an independent workgroup, so a large problem's tiles run side by side.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void batched_emit(int64_t i, int64_t j, float val, int64_t n,
                                             double si, double sj, float* Q, float* q,
                                             bool diag_tile) {
  if (i >= n) return;
  if (j < n) {
    if (diag_tile && i > j) return;
    float out;
    if (i == j) out = val > 0.f ? 1.f : 0.f;
    else out = (float)((double)val / (si * sj));
    Q[i * n + j] = out;
    if (i != j) Q[j * n + i] = out;
  } else if (j == n) {
    q[i] = (float)(-(double)val / si);
  }
}

template <int BM, bool DIAG>
__global__ __launch_bounds__(256) void batched_gram_kernel(const BatchGramItem* __restrict__ items,
                                                           const BatchDesc* __restrict__ desc,
                                                           const float* __restrict__ A_pool,
                                                           const float* __restrict__ B_pool,
                                                           float* __restrict__ Q_pool,
                                                           float* __restrict__ q_pool,
                                                           double* __restrict__ s_pool) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  __shared__ double s_l[BM];
  __shared__ float dg[BM];
  const BatchGramItem it = items[blockIdx.x];
  const BatchDesc D = desc[it.p];
  const int64_t n = D.n, d = D.d;
  const float* A = A_pool + D.offA;
  const float* B = B_pool + D.offB;
  float* Q = Q_pool + D.offQ;
  float* q = q_pool + D.offq;
  const double* sp = s_pool + D.offq;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int MT = BM / 32;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BM / 2);
  const int out_col = lane & 15, out_row = (lane >> 4) * 4;
  const int64_t i0 = (int64_t)it.ti * BM, j0 = (int64_t)it.tj * BM;
  const GramPanelPtr px = panel_column(i0 + tid % BM, n, 1, A, n, B, 1);
  const GramPanelPtr py = panel_column(j0 + tid % BM, n, 1, A, n, B, 1);
  f32x4 acc[MT][MT];
  gram_tile_bf16x3<BM>(acc, 0, d, px, py, DIAG, lds);
  if (DIAG) {
    // diagonal entries of the block -> scales of its rows
    if (wm == wn) {
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int e = out_col - out_row;
#pragma unroll
        for (int ee = 0; ee < 4; ++ee)
          if (ee == e) dg[wm + a * 16 + out_col] = acc[a][a][ee];
      }
    }
    __syncthreads();
    if (tid < BM) {
      const int64_t i = i0 + tid;
      const float h = dg[tid];
      const double si = h > 0.f ? sqrt((double)h) : 1.0;
      s_l[tid] = si;
      if (i < n) s_pool[D.offq + i] = si;
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int li = wm + a * 16 + out_row + e;
      const int64_t i = i0 + li;
      if (i >= n) continue;
      const double si = DIAG ? s_l[li] : sp[i];
#pragma unroll
      for (int b = 0; b < MT; ++b) {
        const int lj = wn + b * 16 + out_col;
        const int64_t j = j0 + lj;
        const double sj = j < n ? (DIAG ? s_l[lj] : sp[j]) : 1.0;
        batched_emit(i, j, acc[a][b][e], n, si, sj, Q, q, DIAG);
      }
    }
}

size_t batched_gram_lds_bytes(int bm) {
  return bm == 64 ? (size_t)GbTile<64>::LDS_BYTES : (size_t)GbTile<128>::LDS_BYTES;
}

hipError_t prepare_batched_gram() {
  hipError_t e = hipSuccess;
  auto set = [&](const void* k, int bytes) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
  set((const void*)batched_gram_kernel<64, true>, GbTile<64>::LDS_BYTES);
  set((const void*)batched_gram_kernel<64, false>, GbTile<64>::LDS_BYTES);
  set((const void*)batched_gram_kernel<128, true>, GbTile<128>::LDS_BYTES);
  set((const void*)batched_gram_kernel<128, false>, GbTile<128>::LDS_BYTES);
  return e;
}

hipError_t launch_batched_gram(int bm, bool diag, const BatchGramItem* items, int64_t count,
                               const BatchDesc* desc, const float* A_pool, const float* B_pool,
                               float* Q_pool, float* q_pool, double* s_pool, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const dim3 grid((unsigned)count), block(256);
  const size_t lds = batched_gram_lds_bytes(bm);
  if (bm == 64) {
    if (diag)
      hipLaunchKernelGGL((batched_gram_kernel<64, true>), grid, block, lds, st, items, desc,
                         A_pool, B_pool, Q_pool, q_pool, s_pool);
    else
      hipLaunchKernelGGL((batched_gram_kernel<64, false>), grid, block, lds, st, items, desc,
                         A_pool, B_pool, Q_pool, q_pool, s_pool);
  } else {
    if (diag)
      hipLaunchKernelGGL((batched_gram_kernel<128, true>), grid, block, lds, st, items, desc,
                         A_pool, B_pool, Q_pool, q_pool, s_pool);
    else
      hipLaunchKernelGGL((batched_gram_kernel<128, false>), grid, block, lds, st, items, desc,
                         A_pool, B_pool, Q_pool, q_pool, s_pool);
  }
  return hipGetLastError();
}

// Sum of the split-K partial tiles in fixed split order and the rescale epilogue.  Block (tile,
// 8-row band of the tile), one thread per column: the band's 8 partial rows of a split are read
// together (coalesced, 8 loads in flight per thread) and the direct write Q[i, j] is coalesced;
// the rescaled band is staged in LDS so that thread jj writes the mirrored Q[j, i] as 8
// consecutive floats of row j.  Same values and rules as gram_emit (s == nullptr: no rescale).
constexpr int GE_BAND = 8;

template <int TILE>
__global__ __launch_bounds__(TILE) void gram_splitk_epilogue_kernel(
    int64_t n, int64_t k, const float* __restrict__ partial, int nsplit, int ntiles,
    int tiles_aug, const double* __restrict__ s, float* __restrict__ Q, float* __restrict__ q) {
  __shared__ float band[GE_BAND][TILE + 1];
  int ti, tj;
  decode_tile(blockIdx.x, tiles_aug, ti, tj);
  const bool diag = (ti == tj);
  const int64_t i0 = (int64_t)ti * TILE + (int64_t)blockIdx.y * GE_BAND, j0 = (int64_t)tj * TILE;
  const int lj = threadIdx.x;
  const int64_t j = j0 + lj;
  const float* src = partial + (int64_t)blockIdx.x * (TILE * TILE) +
                     (int64_t)blockIdx.y * GE_BAND * TILE + lj;
  float acc[GE_BAND];
#pragma unroll
  for (int r = 0; r < GE_BAND; ++r) acc[r] = 0.f;
  for (int sp = 0; sp < nsplit; ++sp) {
    const float* sp_src = src + (int64_t)sp * ntiles * (TILE * TILE);
#pragma unroll
    for (int r = 0; r < GE_BAND; ++r) acc[r] += sp_src[r * TILE];
  }
#pragma unroll
  for (int r = 0; r < GE_BAND; ++r) {
    const int64_t i = i0 + r;
    float out = acc[r];
    if (i < n && j < n) {
      if (s != nullptr)
        out = (i == j) ? (acc[r] > 0.f ? 1.f : 0.f) : (float)((double)acc[r] / (s[i] * s[j]));
      if (!(diag && i > j)) Q[i * n + j] = out;
    } else if (i < n && j < n + k) {
      q[i * k + (j - n)] = s == nullptr ? -acc[r] : (float)(-(double)acc[r] / s[i]);
    }
    band[r][lj] = out;
  }
  __syncthreads();
  // mirror: thread jj writes row j0 + jj, columns i0 .. i0 + 7
  if (j < n) {
#pragma unroll
    for (int r = 0; r < GE_BAND; ++r) {
      const int64_t i = i0 + r;
      if (i < n && i != j && !(diag && i > j)) Q[j * n + i] = band[r][lj];
    }
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
  hipLaunchKernelGGL(colnorm_finalize_kernel, dim3((unsigned)((n + CN_C - 1) / CN_C)), dim3(256),
                     0, st, n, chunks, (const double*)ws, s);
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

// Layout of the single-problem BF16x3 workspace: Ph, Pl (pre-split [A | B]) and, with split-K,
// the partial tiles.
struct GramDmaPlan {
  int tiles_a, tiles_aug, ntiles, splits;
  int64_t dpad, ncols_pad, rows_per_split;
  size_t split_bytes, partial_bytes;
};

static GramDmaPlan gram_dma_plan(int64_t d, int64_t n, int64_t k) {
  GramDmaPlan p;
  gram_tiles(n, k, GD_T, p.tiles_a, p.tiles_aug, p.ntiles);
  p.dpad = (d + PS_T - 1) / PS_T * PS_T;
  p.ncols_pad = (int64_t)p.tiles_aug * GD_T;
  // One workgroup per compute unit, 256 at a time: split the rows of A into s parts where
  // that shortens the critical path, rounds(s) / s with rounds = ceil(tiles * s / 256), with a
  // small charge per split for the partial tiles; each part keeps at least 8 K steps.
  int64_t max_splits = p.dpad / (8 * GD_BK);
  if (max_splits > 16) max_splits = 16;
  int splits = 1;
  double best = 1e30;
  for (int sp = 1; sp <= (max_splits > 1 ? max_splits : 1); ++sp) {
    const double rounds = (double)(((int64_t)p.ntiles * sp + 255) / 256);
    const double cost = rounds / sp * (1.0 + 0.05 * sp);
    if (cost < best) {
      best = cost;
      splits = sp;
    }
  }
  int64_t rows = (p.dpad + splits - 1) / splits;
  rows = (rows + GD_BK - 1) / GD_BK * GD_BK;
  p.splits = (int)((p.dpad + rows - 1) / rows);
  p.rows_per_split = rows;
  p.split_bytes = sizeof(uint16_t) * (size_t)p.ncols_pad * (size_t)p.dpad;
  p.partial_bytes = p.splits > 1 ? sizeof(float) * (size_t)p.splits * p.ntiles * GD_T * GD_T : 0;
  return p;
}


size_t gram_bf16x3_ws_bytes(int64_t d, int64_t n, int64_t k) {
  const GramDmaPlan p = gram_dma_plan(d, n, k);
  return 2 * p.split_bytes + p.partial_bytes;
}

// The operand split: [A | B] -> column-major BF16 hi / lo planes in ws.  With s_out !=
// nullptr it also forms the column norms (partials in colsq) and writes them to s_out.
static hipError_t split_bf16x3(const GramDmaPlan& p, int64_t d, int64_t n, int64_t k,
                               const float* A, int64_t lda, const float* B, int64_t ldb,
                               float* ws, double* colsq, double* s_out, hipStream_t st) {
  uint16_t* Ph = (uint16_t*)ws;
  uint16_t* Pl = (uint16_t*)((char*)ws + p.split_bytes);
  dim3 g0((unsigned)(p.ncols_pad / PS_T), (unsigned)(p.dpad / PS_T));
  hipLaunchKernelGGL(presplit_kernel, g0, dim3(256), 0, st, d, n, k, A, lda, B, ldb, p.dpad, Ph,
                     Pl, s_out != nullptr ? colsq : nullptr);
  if (s_out != nullptr)
    hipLaunchKernelGGL(colnorm_finalize_kernel, dim3((unsigned)((n + CN_C - 1) / CN_C)),
                       dim3(256), 0, st, n, p.dpad / PS_T, (const double*)colsq, s_out);
  return hipGetLastError();
}

// The matrix-core product from the planes in ws, with the rescale by s (or none) in the
// epilogue (through the split-K partials in ws when the plan splits K).
static hipError_t product_bf16x3(const GramDmaPlan& p, int64_t n, int64_t k, const double* s,
                                 float* Q, float* q, float* ws, hipStream_t st) {
  const uint16_t* Ph = (const uint16_t*)ws;
  const uint16_t* Pl = (const uint16_t*)((char*)ws + p.split_bytes);
  float* partial = p.splits > 1 ? (float*)((char*)ws + 2 * p.split_bytes) : nullptr;
  const int blocks = schedule_blocks(p.ntiles, p.splits);
  hipError_t e = hipFuncSetAttribute((const void*)gram_dma_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, GD_LDS_BYTES);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_dma_kernel, dim3((unsigned)blocks), dim3(GD_NT), GD_LDS_BYTES, st, n, k,
                     Ph, Pl, p.dpad, s, Q, q, partial, p.tiles_a, p.tiles_aug, p.ntiles,
                     p.splits, p.rows_per_split);
  if (p.splits > 1)
    hipLaunchKernelGGL(gram_splitk_epilogue_kernel<GD_T>,
                       dim3((unsigned)p.ntiles, GD_T / GE_BAND), dim3(GD_T), 0, st, n, k,
                       (const float*)partial, p.splits, p.ntiles, p.tiles_aug, s, Q, q);
  return hipGetLastError();
}

hipError_t launch_gram_bf16x3(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                              const float* B, int64_t ldb, const double* s, float* Q, float* q,
                              float* ws, hipStream_t st) {
  const GramDmaPlan p = gram_dma_plan(d, n, k);
  hipError_t e = split_bf16x3(p, d, n, k, A, lda, B, ldb, ws, nullptr, nullptr, st);
  if (e != hipSuccess) return e;
  return product_bf16x3(p, n, k, s, Q, q, ws, st);
}

size_t prepare_bf16x3_ws_bytes(int64_t d, int64_t n, int64_t k) {
  const GramDmaPlan p = gram_dma_plan(d, n, k);
  const size_t gram = (2 * p.split_bytes + p.partial_bytes + 255) / 256 * 256;
  return gram + sizeof(double) * (size_t)(p.dpad / PS_T) * (size_t)n;
}

hipError_t launch_prepare_split_bf16x3(int64_t d, int64_t n, int64_t k, const float* A,
                                       int64_t lda, const float* B, int64_t ldb, double* s,
                                       void* ws, hipStream_t st) {
  const GramDmaPlan p = gram_dma_plan(d, n, k);
  const size_t gram = (2 * p.split_bytes + p.partial_bytes + 255) / 256 * 256;
  double* colsq = (double*)((char*)ws + gram);
  return split_bf16x3(p, d, n, k, A, lda, B, ldb, (float*)ws, colsq, s, st);
}

hipError_t launch_prepare_product_bf16x3(int64_t d, int64_t n, int64_t k, const double* s,
                                         float* Q, float* q, void* ws, hipStream_t st) {
  return product_bf16x3(gram_dma_plan(d, n, k), n, k, s, Q, q, (float*)ws, st);
}

hipError_t launch_prepare_bf16x3(int64_t d, int64_t n, int64_t k, const float* A, int64_t lda,
                                 const float* B, int64_t ldb, double* s, float* Q, float* q,
                                 void* ws, hipStream_t st) {
  hipError_t e = launch_prepare_split_bf16x3(d, n, k, A, lda, B, ldb, s, ws, st);
  if (e != hipSuccess) return e;
  return launch_prepare_product_bf16x3(d, n, k, s, Q, q, ws, st);
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
