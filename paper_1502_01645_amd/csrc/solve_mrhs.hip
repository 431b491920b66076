// Algorithm 2 for many right-hand sides sharing Q (an NMF-style update: small n, large k).
//
// A workgroup owns 16 column slots.  Per update, for all its active columns at once:
//   gbar = masked gradient (passive set per column), num_c = ||gbar_c||^2, residual r_c;
//   W = Q * Gbar on the FP32 matrix cores: 16 output columns.  For n <= 256 Q is held in the
//   registers of each workgroup (v_mfma_f32_16x16x4f32 for 16 slots; v_mfma_f32_4x4x1f32 passes
//   of 4 slots when at most 8 update), or on request as FP16 hi and lo parts with the three-term
//   split Q_lo V_hi + Q_hi V_lo + Q_hi V_hi on v_mfma_f32_16x16x32_f16 (below); for n > 256 Q is
//   read from L2 (every workgroup streams the same n x n matrix) for v_mfma_f32_16x16x4f32;
//   den_c = gbar_c^T W_c, alpha_c = num_c / den_c;  y' = [y - alpha gbar]_+;
//   grad' = grad + Q (y' - y), the second product of Algorithm 2, again on the matrix cores
//   (with 16 columns per product the full product beats gathering the clipped rows of Q).
// A column whose residual meets tol has its gradient recomputed exactly (Q y + q, one more
// matrix-core product, always on the FP32 Q) before it retires; it then writes x = y / s, its
// iteration count, residual and status, and the slot takes the next column from a queue.
// State lives in LDS as [row][slot] arrays; rows are padded to a multiple of 16.
#include <stdlib.h>
#include <string.h>

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int MR_NT = 256;
constexpr int MR_SLOTS = 16;

// v[l] + v[l ^ 16] and v[l] + v[l ^ 32] for every lane l, on the vector ALU (the LDS crossbar of
// a lane shuffle costs a round trip).  v_permlane16_swap_b32 exchanges the odd 16-lane rows of
// its first register with the even rows of its second, v_permlane32_swap_b32 the upper 32 lanes
// of its first with the lower 32 of its second: applied to two copies of v, the two registers
// then hold the lower and the upper value of each lane's pair, and their sum is bitwise the same
// in both lanes of the pair.  Every lane must be active.  (s_nop 1: the swap reads registers that
// the instructions just before may have written.)
__device__ __forceinline__ float add_xor16(float v) {
  float a = v, b = v;
  asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  return a + b;
}
__device__ __forceinline__ float add_xor32(float v) {
  float a = v, b = v;
  asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  return a + b;
}

// Line-search denominators from a product's epilogue: den_c = V_c^T W_c, summed per lane over
// the output entries it writes (Vd[row][c] * W[row][c]), then over the four lanes of the wave
// that share the slot; lanes 0..15 of each wave write the wave's partial to redw[wave][slot].
// Every wave calls it (with 0 when it wrote nothing).  Products that form no denominator are
// instantiated with DEN = false and leave redw alone.
__device__ __forceinline__ void den_publish(float dp, float* redw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  dp = add_xor32(add_xor16(dp));
  // (the index is formed here each time rather than kept in a register through the solve)
  int at = wave * MR_SLOTS + lane;
  asm volatile("" : "+v"(at));
  if (lane < MR_SLOTS) redw[at] = dp;
}

// Split products for Q held in registers (the form NNLS_MRHS_PRODUCT=split16 selects; the
// default products are FP32).  A value x in FP32 is written as hi + lo with
// hi = fp16(x) and lo = fp16(x - hi): both are FP16 (11-bit significands), so |x - hi - lo| is
// at most 2^-22 |x| (the rounding of lo) as long as lo stays in FP16's normal range, and the
// dropped term lo_Q lo_V is at most 2^-22 |Q_ij V_j|.  The products are exact in the matrix
// core and summed in FP32, so each term of Q V carries at most 3 2^-22 relative error, against
// the 2^-24 roundings of the FP32 product's sums.  That is close enough for the two products of
// an update, which steer the iteration; the exact gradient that decides the stop test, where
// Q y and q nearly cancel, is formed from the FP32 Q instead.  To keep both parts in FP16's
// range every row i of Q is scaled by a power of two r_i that brings its largest entry to
// [2^13, 2^14), and every column c of the vector operand by a power
// of two sigma_c from a bound on its largest entry (the slot's ||gbar|| or alpha ||gbar||);
// W = (scaled product) / (r_i sigma_c) exactly.  One v_mfma_f32_16x16x32_f16 (16
// cycles) covers the k range of eight v_mfma_f32_16x16x4f32 (32 cycles each), so the three
// split products take 3/16 of the matrix-core time of the FP32 product.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
constexpr int MR_H3_EXP = 14;  // scaled entries stay below 2^14 (FP16 max is 65504)

// sigma with bound * sigma in [2^13, 2^14): a power of two, 1 for a bound that is 0 or not
// finite
__device__ __forceinline__ float mr_pow2_scale(float bound) {
  if (!(bound > 0.f) || !__builtin_isfinite(bound)) return 1.f;
  int e = 0;
  (void)frexpf(bound, &e);  // bound = m 2^e, m in [0.5, 1)
  int x = MR_H3_EXP - e;
  x = x < -126 ? -126 : (x > 126 ? 126 : x);
  return ldexpf(1.f, x);
}

// FP16 hi and lo parts of 8 consecutive rows of one column, scaled by sig, as one entry of the
// B operand of v_mfma_f32_16x16x32_f16: entry 16 rb + c of Vh / Vl holds rows 8 rb + 0..7 of
// column c (so k block kh, lane l of a product reads entry 64 kh + l: rows 32 kh + 8 (l / 16) +
// 0..7 of column l % 16).
__device__ __forceinline__ void split_chunk(const float (&v)[8], float sig, f16x8* h_out,
                                            f16x8* l_out) {
  f16x8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = v[e] * sig;
    const _Float16 hx = (_Float16)x;
    h[e] = hx;
    l[e] = (_Float16)(x - (float)hx);
  }
  *h_out = h;
  *l_out = l;
}

// W = Q * V from the register-held split Q (rows scaled by r, rinv = 1 / r in LDS) and the split
// V (columns scaled by sigma; cs = 1 / sigma of the lane's column): wave w owns the row tiles
// w + NW tt, lane l holds rows 16 t + l % 16 at columns 32 kh + 8 (l / 16) + 0..7 (the A
// operand).  W is [np][S] and Vd [np][SV] in LDS.
template <int TW, int KH, int NW, int S, bool DEN, int SV = S>
__device__ __forceinline__ void mfma_product_h3(const f16x8 (&qh)[TW][KH],
                                                const f16x8 (&ql)[TW][KH], const f16x8* Vh,
                                                const f16x8* Vl, const float* rinv, float cs,
                                                float* W, const float* Vd, float* redw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  f32x4 acc[TW];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) acc[tt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kh = 0; kh < KH; ++kh) {
    const f16x8 bh = Vh[kh * 64 + lane], bl = Vl[kh * 64 + lane];
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) {
      acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ql[tt][kh], bh, acc[tt], 0, 0, 0);
      acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qh[tt][kh], bl, acc[tt], 0, 0, 0);
      acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qh[tt][kh], bh, acc[tt], 0, 0, 0);
    }
  }
  float dp = 0.f;
  // the lane's first output row, formed here rather than kept in a register through the solve;
  // the other rows are constant offsets from it
  int row0 = wave * 16 + 4 * lg;
  asm volatile("" : "+v"(row0));
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = row0 + NW * 16 * tt + e;
      const float w = (acc[tt][e] * rinv[row]) * cs;
      W[row * S + lr] = w;
      if constexpr (DEN) dp += Vd[row * SV + lr] * w;
    }
  }
  if constexpr (DEN) den_publish(dp, redw);
}

struct MrArgs {
  int n, np, k;
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
  float* trace;  // [k][trace_len][2] per-update record (r, ||gbar||^2), or nullptr
  int trace_len;
  int* queue;  // next unassigned column (starts at 16 * gridDim.x)
  const float* G0;  // [n, k] exact gradients Q max(Y0, 0) + q at the start, or nullptr
};

// W[0..np)[0..16) = Q * V (V and Vd: [np][16] in LDS, rows SV floats apart; W rows S floats
// apart), rows and columns of Q
// beyond n read as 0.
// Wave w computes row tiles w, w + NT / 64, ...; for each 16-wide k block a lane loads 4
// consecutive Q entries of one row (16 bytes) and feeds them to 4 MFMAs; the k index of MFMA e
// for lane group g is k0 + 4 g + e, for both operands.  KB k blocks (8 by default) are loaded
// before their MFMAs so the L2 latency is paid once per KB.
template <int NT, bool DEN, int KB = 8, int S = MR_SLOTS, int SV = S>
__device__ void mfma_product(const MrArgs& A, const float* V, float* W, const float* Vd,
                             float* redw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = A.n, np = A.np;
  const int tiles = np / 16;
  const int lr = lane & 15, lg = lane >> 4;
  float dp = 0.f;
  // KB: k blocks (of 16) whose Q fragments are in flight together
  for (int t = wave; t < tiles; t += NT / kWave) {
    const int m = t * 16 + lr;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* qrow = A.Q + (int64_t)m * n;
    for (int k0 = 0; k0 < np; k0 += 16 * KB) {
      f32x4 a[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int kk = k0 + 16 * u + 4 * lg;
        a[u] = (m < n && kk < n) ? *(const f32x4*)(qrow + kk) : (f32x4){0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int kk = k0 + 16 * u + 4 * lg;
        if (k0 + 16 * u < np) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float b = V[(kk + e) * SV + lr];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][e], b, acc, 0, 0, 0);
          }
        }
      }
    }
    // D layout: lane holds column (lane & 15), rows 4 * (lane >> 4) + e of the tile
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = t * 16 + 4 * lg + e;
      W[row * S + lr] = acc[e];
      if constexpr (DEN) dp += Vd[row * SV + lr] * acc[e];
    }
  }
  if constexpr (DEN) den_publish(dp, redw);
}

// Start gradients of a warm-started solve, G0 = Q max(Y0, 0) + q, for every column at once:
// the exact gradient the solver would otherwise form for each slot group whenever a column
// enters a slot.  One workgroup per 16 columns: their max(Y0, 0) staged in LDS, the product on
// the FP32 matrix cores with Q read from L2 (mfma_product, the solver's own exact-gradient
// arithmetic), q added in the write-out.  np <= 256.
constexpr int SG_NP = 256;
__global__ __launch_bounds__(MR_NT) void mrhs_start_grad_kernel(MrArgs A, float* G0) {
  __shared__ float V[SG_NP * MR_SLOTS];
  __shared__ float Wt[SG_NP * MR_SLOTS];
  const int n = A.n, np = A.np, k = A.k;
  const int64_t c0 = (int64_t)blockIdx.x * MR_SLOTS;
  for (int e = threadIdx.x; e < np * MR_SLOTS; e += MR_NT) {
    const int i = e / MR_SLOTS;
    const int64_t col = c0 + e % MR_SLOTS;
    float v = 0.f;
    if (i < n && col < k) {
      v = A.Y0[(int64_t)i * k + col];
      v = v > 0.f ? v : 0.f;  // the solver's own reading of a start entry
    }
    V[e] = v;
  }
  __syncthreads();
  mfma_product<MR_NT, false>(A, V, Wt, nullptr, nullptr);
  __syncthreads();
  for (int e = threadIdx.x; e < np * MR_SLOTS; e += MR_NT) {
    const int i = e / MR_SLOTS;
    const int64_t col = c0 + e % MR_SLOTS;
    if (i < n && col < k) G0[(int64_t)i * k + col] = Wt[e] + A.q[(int64_t)i * k + col];
  }
}

// W = Q * V with Q held in registers (n <= 256): of NW waves, wave w owns the row tiles
// t = w + NW tt (tt < TW); lane l holds Q[16 t + l % 16][4 ks + l / 16] for every k step
// ks < KS (np = 4 KS), the A operand of MFMA ks, so a product reads only V from LDS (lane l: row
// 4 ks + l / 16, slot l % 16; 16 consecutive lanes hit 16 consecutive banks) and one V value
// feeds TW MFMAs.  V and Vd rows are SV floats apart, W rows S.
template <int TW, int KS, int NW, bool DEN, int S = MR_SLOTS, int SV = S>
__device__ __forceinline__ void mfma_product_reg(const float (&qa)[TW][KS], const float* V,
                                                 float* W, const float* Vd, float* redw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  f32x4 acc[TW];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) acc[tt] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // (the V values of the next 4 steps are read while the current 4 are multiplied)
  constexpr int KC = 4;
  static_assert(KS % KC == 0, "k steps per chunk");
  float bn[KC];
#pragma unroll
  for (int u = 0; u < KC; ++u) bn[u] = V[(4 * u + lg) * SV + lr];
#pragma unroll
  for (int k0 = 0; k0 < KS; k0 += KC) {
    float bc[KC];
#pragma unroll
    for (int u = 0; u < KC; ++u) bc[u] = bn[u];
    if (k0 + KC < KS)
#pragma unroll
      for (int u = 0; u < KC; ++u) bn[u] = V[(4 * (k0 + KC + u) + lg) * SV + lr];
    __builtin_amdgcn_sched_barrier(0);  // (keeps the reads ahead of the products)
#pragma unroll
    for (int u = 0; u < KC; ++u)
#pragma unroll
      for (int tt = 0; tt < TW; ++tt)
        acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[tt][k0 + u], bc[u], acc[tt], 0, 0, 0);
  }
  float dp = 0.f;
  // (the first output row formed here, not kept in a register through the solve)
  int row0 = wave * 16 + 4 * lg;
  asm volatile("" : "+v"(row0));
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = row0 + NW * 16 * tt + e;
      W[row * S + lr] = acc[tt][e];
      if constexpr (DEN) dp += Vd[row * SV + lr] * acc[tt][e];
    }
  }
  if constexpr (DEN) den_publish(dp, redw);
}

// W = Q V for the columns of V whose bits are set in `live` (at most 4 npass of them), with Q in
// registers as for mfma_product_reg, on v_mfma_f32_4x4x1f32: that instruction treats the wave
// as 16 blocks b = l / 4 of 4 x 4, lane 4 b + i giving row i of the A block and lane 4 b + j
// column j of the B block, and lane 4 b + j receiving column j of the block's result (row i in
// element i).  Lane l's Q value for step ks (row 16 t + l % 16, column 4 ks + l / 16) thus
// makes block b a 4-row piece of the tile (rows 16 t + 4 (b % 4) + i) at one column k = 4 ks +
// b / 4, and lane 4 b + j supplies V[k][slot j]: each block accumulates the k of one residue
// mod 4 for 4 slots, and the four residues (lane groups l / 16) are summed by two shuffles.  A
// pass covers 4 slots at a quarter of the matrix-core time of the 16-slot product.  Results of
// other columns are not written; with DEN, the partial denominators of the live slots only.
template <int TW, int KS, int NW, bool DEN, int S, int SV>
__device__ __forceinline__ void mfma_product_few(const float (&qa)[TW][KS], const float* V,
                                                 float* W, const float* Vd, float* redw,
                                                 unsigned live, int npass) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4, j = lane & 3;
  for (int p = 0; p < npass; ++p) {
    // the lane's slot: the (4 p + j)-th set bit of live, or -1 past the last
    int slot = -1;
    {
      unsigned m = live;
      for (int skip = 4 * p + j; skip > 0 && m; --skip) m &= m - 1u;
      if (m) slot = __builtin_ctz(m);
    }
    const int sv = slot < 0 ? 0 : slot;  // (a lane without a slot computes a column never written)
    f32x4 acc[TW];
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) acc[tt] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // (the V values of the next 8 steps are read while the current 8 are multiplied: a step
    // here is too short to cover the LDS latency by itself)
    constexpr int KC = 8;
    static_assert(KS % KC == 0, "k steps per chunk");
    float bn[KC];
#pragma unroll
    for (int u = 0; u < KC; ++u) bn[u] = V[(4 * u + lg) * SV + sv];
#pragma unroll
    for (int k0 = 0; k0 < KS; k0 += KC) {
      float bc[KC];
#pragma unroll
      for (int u = 0; u < KC; ++u) bc[u] = bn[u];
      if (k0 + KC < KS)
#pragma unroll
        for (int u = 0; u < KC; ++u) bn[u] = V[(4 * (k0 + KC + u) + lg) * SV + sv];
      __builtin_amdgcn_sched_barrier(0);  // (keeps the reads ahead of the products)
#pragma unroll
      for (int u = 0; u < KC; ++u)
#pragma unroll
        for (int tt = 0; tt < TW; ++tt)
          acc[tt] = __builtin_amdgcn_mfma_f32_4x4x1f32(qa[tt][k0 + u], bc[u], acc[tt], 0, 0, 0);
    }
    float dp = 0.f;
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[tt][e] = add_xor32(add_xor16(acc[tt][e]));
      }
      // every lane group holds the sums: group g writes row 4 (l % 16 / 4) + g of the tile
      const float w = lg == 0 ? acc[tt][0] : lg == 1 ? acc[tt][1] : lg == 2 ? acc[tt][2] : acc[tt][3];
      const int row = (wave + NW * tt) * 16 + 4 * (lr >> 2) + lg;
      if (slot >= 0) {
        W[row * S + slot] = w;
        if constexpr (DEN) dp += Vd[row * SV + slot] * w;
      }
    }
    if constexpr (DEN) {
      // the wave's partial for slot j of the pass: the 16 lanes with l % 4 == j
      dp += __shfl_xor(dp, 4, 64);
      dp += __shfl_xor(dp, 8, 64);
      dp = add_xor32(add_xor16(dp));
      if (lane < 4 && slot >= 0) redw[wave * MR_SLOTS + slot] = dp;
    }
  }
}

// n > 256: Q does not fit in registers and every product reads it from L2 (mfma_product, FP32).
// Slot state in LDS; threads 0..15 take the slots' decisions and wave 0 folds the slot flags
// into masks.  (n <= 256 runs solve_mrhs_reg_kernel below.)
template <int NT>
__global__ __launch_bounds__(NT, 2) void solve_mrhs_kernel(MrArgs A) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  const int np = A.np, n = A.n;
  float* Y = sm;                       // [np][16]
  float* Gr = Y + np * MR_SLOTS;       // [np][16] gradient
  float* P = Gr + np * MR_SLOTS;       // [np][16] masked gradient / product operand
  float* W = P + np * MR_SLOTS;        // [np][16] product result
  float* colf = W + np * MR_SLOTS;     // per-slot floats [8][16]
  int* coli = (int*)(colf + 8 * MR_SLOTS);  // per-slot ints [9][16]
  float* red = (float*)(coli + 9 * MR_SLOTS);  // [NT / 64 waves][16 slots][4]
  int* s_anyclip = (int*)(red + (NT / kWave) * MR_SLOTS * 4);  // some slot clipped this update
  // bit masks over the slots, rebuilt by wave 0 whenever the slot flags change: live (holds a
  // column), act (takes an update this pass), ref (needs an exact gradient), done (retired)
  int* s_mask = s_anyclip + 1;  // [4]
  enum { M_LIVE = 0, M_ACT = 1, M_REF = 2, M_DONE = 3 };

  // per-slot state in LDS
  float* s_num = colf + 0 * MR_SLOTS;
  float* s_res = colf + 1 * MR_SLOTS;
  float* s_alpha = colf + 2 * MR_SLOTS;
  float* s_qn = colf + 3 * MR_SLOTS;      // ||q_c|| (1 if 0)
  float* s_den = colf + 4 * MR_SLOTS;
  float* s_cnt = colf + 5 * MR_SLOTS;     // passive count
  float* s_bad = colf + 6 * MR_SLOTS;
  int* s_col = coli + 0 * MR_SLOTS;       // column id or -1
  int* s_it = coli + 1 * MR_SLOTS;        // updates done
  int* s_fresh = coli + 2 * MR_SLOTS;     // gradient exact since last update
  int* s_act = coli + 3 * MR_SLOTS;       // take an update this pass
  int* s_ref = coli + 4 * MR_SLOTS;       // needs an exact gradient
  int* s_rows = coli + 5 * MR_SLOTS;      // rows of Q read (low bits)
  int* s_rowsh = coli + 6 * MR_SLOTS;     // rows of Q read (high bits)
  int* s_done = coli + 7 * MR_SLOTS;      // outputs written; slot waits for a new column
  int* s_clip = coli + 8 * MR_SLOTS;      // clipped rows of the gradient corrections so far

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int slot = tid & 15;              // elementwise mapping: slot = tid % 16,
  const int row0 = tid >> 4;              // rows row0 + 16 m

  // W = Q V for V [np][16] in LDS; with den, also the partials of V_c^T W_c per wave and slot
  // in red[wave][slot]
  auto product = [&](const float* V, float* Wout, auto den) {
    constexpr bool DEN = decltype(den)::value;
    mfma_product<NT, DEN>(A, V, Wout, V, red);
  };

  // The slot flags are written by threads 0..15 (lanes 0..15 of wave 0).  Wave 0 then folds
  // them into s_mask with ballots; the caller's next barrier makes the masks visible, and every
  // other thread reads one word instead of sixteen flags.
  auto publish_masks = [&]() {
    if (wave == 0) {
      __builtin_amdgcn_wave_barrier();
      const bool in = lane < MR_SLOTS;
      const bool live = in && s_col[lane] >= 0;
      const unsigned long long mlive = __ballot(live);
      const unsigned long long mact = __ballot(in && s_act[lane] != 0);
      const unsigned long long mref = __ballot(live && s_ref[lane] != 0);
      const unsigned long long mdone = __ballot(live && s_done[lane] != 0);
      if (lane == 0) {
        s_mask[M_LIVE] = (int)mlive;
        s_mask[M_ACT] = (int)mact;
        s_mask[M_REF] = (int)mref;
        s_mask[M_DONE] = (int)mdone;
      }
    }
  };

  // -- load a column into a slot: y = max(Y0, 0) or 0, gradient = q (exact for a cold start)
  auto load_slot = [&](int sl, int col) {
    // called by the 16 threads of slot sl (tid % 16 == sl)
    for (int i = row0; i < np; i += NT / MR_SLOTS) {
      float qi = 0.f, yi = 0.f;
      if (col >= 0 && i < n) {
        qi = A.q[(int64_t)i * A.k + col];
        if (A.Y0) {
          yi = A.Y0[(int64_t)i * A.k + col];
          yi = yi > 0.f ? yi : 0.f;
        }
      }
      Y[i * MR_SLOTS + sl] = yi;
      Gr[i * MR_SLOTS + sl] = qi;
    }
  };

  if (tid < MR_SLOTS) {
    const int col = blockIdx.x * MR_SLOTS + tid;
    s_col[tid] = col < A.k ? col : -1;
    s_it[tid] = 0;
    s_fresh[tid] = A.Y0 ? 0 : 1;
    s_ref[tid] = A.Y0 ? 1 : 0;
    s_rows[tid] = 0;
    s_rowsh[tid] = 0;
    s_done[tid] = 0;
    s_clip[tid] = 0;
    s_act[tid] = 0;
    if (tid == 0) *s_anyclip = 0;
  }
  publish_masks();
  __syncthreads();
  load_slot(slot, s_col[slot]);
  __syncthreads();

  // per-slot reduction of four per-thread values over the 16 threads sharing a slot
  // (sync_after = false leaves out the trailing barrier: only threads 0..15 may then read the
  // results, each its own slot's)
  auto slot_reduce4 = [&](float v0, float v1, float v2, float v3, float* o0, float* o1,
                          float* o2, float* o3, bool sync_after = true) {
    // lanes with equal (lane & 15) share a slot within a wave: xor 16, 32
    v0 = add_xor32(add_xor16(v0));
    v1 = add_xor32(add_xor16(v1));
    v2 = add_xor32(add_xor16(v2));
    v3 = add_xor32(add_xor16(v3));
    if (lane < 16) {
      float* r = red + (wave * MR_SLOTS + lane) * 4;
      r[0] = v0;
      r[1] = v1;
      r[2] = v2;
      r[3] = v3;
    }
    __syncthreads();
    if (tid < MR_SLOTS) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int w = 0; w < NT / kWave; ++w) {
        const float* r = red + (w * MR_SLOTS + tid) * 4;
        a0 += r[0];
        a1 += r[1];
        a2 += r[2];
        a3 += r[3];
      }
      if (o0) o0[tid] = a0;
      if (o1) o1[tid] = a1;
      if (o2) o2[tid] = a2;
      if (o3) o3[tid] = a3;
    }
    if (sync_after) __syncthreads();
  };

  // ||q_c|| of every slot
  auto slot_qnorm = [&]() {
    float acc = 0.f;
    const int col = s_col[slot];
    if (col >= 0)
      for (int i = row0; i < n; i += NT / MR_SLOTS) {
        const float qi = A.q[(int64_t)i * A.k + col];
        acc += qi * qi;
      }
    slot_reduce4(acc, 0.f, 0.f, 0.f, s_qn, nullptr, nullptr, nullptr);
    if (tid < MR_SLOTS) s_qn[tid] = s_qn[tid] > 0.f ? sqrtf(s_qn[tid]) : 1.f;
    __syncthreads();
  };
  slot_qnorm();

  for (;;) {
    // ---- exact gradient for slots that asked for it: W = Q Y, grad = W + q
    if (s_mask[M_REF]) {
      for (int e = tid; e < np * MR_SLOTS; e += NT) P[e] = Y[e];
      __syncthreads();
      product(P, W, std::false_type{});
      __syncthreads();
      if (s_ref[slot] && s_col[slot] >= 0) {
        const int col = s_col[slot];
        for (int i = row0; i < n; i += NT / MR_SLOTS)
          Gr[i * MR_SLOTS + slot] = W[i * MR_SLOTS + slot] + A.q[(int64_t)i * A.k + col];
      }
      __syncthreads();
      if (tid < MR_SLOTS && s_ref[tid] && s_col[tid] >= 0) {
        s_ref[tid] = 0;
        s_fresh[tid] = 1;
        const unsigned r = (unsigned)s_rows[tid] + (unsigned)n;
        if (r < (unsigned)s_rows[tid]) s_rowsh[tid] += 1;
        s_rows[tid] = (int)r;
      }
      publish_masks();
      __syncthreads();
    }

    // ---- passive set, masked gradient, statistics
    {
      float num = 0.f, res = 0.f, cnt = 0.f, bad = 0.f;
      const bool live = s_col[slot] >= 0;
      for (int i = row0; i < np; i += NT / MR_SLOTS) {
        const int e = i * MR_SLOTS + slot;
        const float yi = Y[e], gi = Gr[e];
        const bool valid = live && i < n;
        const bool pas = valid && ((yi > 0.f) || (gi < 0.f));
        const float pi = pas ? gi : 0.f;
        P[e] = pi;
        num += pi * pi;
        const float m = yi < gi ? yi : gi;
        res += valid ? m * m : 0.f;
        cnt += pas ? 1.f : 0.f;
        bad += (valid && (!__builtin_isfinite(yi) || !__builtin_isfinite(gi))) ? 1.f : 0.f;
      }
      slot_reduce4(num, res, cnt, bad, s_num, s_res, s_cnt, s_bad, false);
    }

    // ---- per-slot decisions (threads 0..15, right after they summed their slot's statistics):
    // finish, refresh, or update
    if (tid < MR_SLOTS) {
      s_act[tid] = 0;
      // the clip flag was last read before the barriers of the statistics reduction
      if (tid == 0) *s_anyclip = 0;
      const int col = s_col[tid];
      if (col >= 0 && !s_done[tid]) {
        const double r = sqrt((double)s_res[tid]) / (double)s_qn[tid];
        if (A.trace != nullptr && s_it[tid] < A.trace_len) {
          float* tr = A.trace + ((int64_t)col * A.trace_len + s_it[tid]) * 2;
          tr[0] = (float)r;
          tr[1] = s_num[tid];
        }
        int st = -1;
        if (s_bad[tid] > 0.f) {
          st = NNLS_NONFINITE_DEV;
        } else if (s_cnt[tid] == 0.f || r <= A.tol) {
          if (s_fresh[tid]) st = NNLS_CONVERGED_DEV;
          else s_ref[tid] = 1;
        } else if (s_it[tid] >= A.max_iter) {
          if (s_fresh[tid]) st = NNLS_MAXITER_DEV;
          else s_ref[tid] = 1;
        } else {
          s_act[tid] = 1;
        }
        if (st >= 0) {
          A.iters[col] = s_it[tid];
          A.kkt[col] = st == NNLS_NONFINITE_DEV ? __builtin_nan("") : r;
          A.status[col] = st;
          if (A.rows_read)
            A.rows_read[col] =
                (((int64_t)s_rowsh[tid] << 32) | (int64_t)(unsigned)s_rows[tid]) + s_clip[tid];
          s_done[tid] = 1;
        }
      }
    }
    publish_masks();
    __syncthreads();
    if (s_mask[M_DONE]) {
      // write x = y / s of finished slots, then give each a new column from the queue
      const bool fin = s_col[slot] >= 0 && s_done[slot];
      if (fin) {
        const int col = s_col[slot];
        for (int i = row0; i < n; i += NT / MR_SLOTS) {
          const float yi = Y[i * MR_SLOTS + slot];
          A.X[(int64_t)i * A.k + col] = A.s ? (float)((double)yi / A.s[i]) : yi;
        }
      }
      __syncthreads();
      if (tid < MR_SLOTS && fin) {
        const int next = atomicAdd(A.queue, 1);
        s_col[tid] = next < A.k ? next : -1;
        s_it[tid] = 0;
        s_done[tid] = 0;
        s_fresh[tid] = A.Y0 ? 0 : 1;
        s_ref[tid] = (A.Y0 && next < A.k) ? 1 : 0;
        s_rows[tid] = 0;
        s_rowsh[tid] = 0;
        s_clip[tid] = 0;
      }
      publish_masks();
      __syncthreads();
      if (fin) load_slot(slot, s_col[slot]);
      __syncthreads();
      slot_qnorm();
      continue;  // evaluate the new columns before any update
    }
    if (!s_mask[M_LIVE]) break;   // every slot empty: the queue is exhausted
    if (!s_mask[M_ACT]) continue;  // only exact-gradient refreshes are pending

    // ---- W = Q Gbar on the matrix cores, with den_c = gbar_c^T W_c from its epilogue.  The
    // columns of W are independent, so the columns of slots that take no update need no
    // clearing: their W is never used.  (P was written before the barrier of the statistics
    // reduction; W and red were last read before the barrier after the decisions.)
    product(P, W, std::true_type{});
    __syncthreads();
    if (tid < MR_SLOTS && s_act[tid]) {
      float den = 0.f;
#pragma unroll
      for (int w = 0; w < NT / kWave; ++w) den += red[w * MR_SLOTS + tid];
      s_den[tid] = den;
      if (!(den > 0.f) || !__builtin_isfinite(den)) {
        // breakdown: retire the column with its current iterate
        const int col = s_col[tid];
        A.iters[col] = s_it[tid];
        A.kkt[col] = sqrt((double)s_res[tid]) / (double)s_qn[tid];
        A.status[col] = NNLS_BREAKDOWN_DEV;
        if (A.rows_read)
          A.rows_read[col] =
              (((int64_t)s_rowsh[tid] << 32) | (int64_t)(unsigned)s_rows[tid]) + s_clip[tid];
        s_act[tid] = 0;
        s_done[tid] = 1;
        s_ref[tid] = 0;
      } else {
        s_alpha[tid] = s_num[tid] / den;
      }
    }
    publish_masks();
    __syncthreads();

    // ---- projected update y' = [y - alpha gbar]_+; P becomes d = y' - y
    int clip_mine = 0;
    {
      const bool act = s_act[slot];
      const float alpha = act ? s_alpha[slot] : 0.f;
      for (int i = row0; i < np; i += NT / MR_SLOTS) {
        const int e = i * MR_SLOTS + slot;
        float d = 0.f;
        if (act && i < n) {
          const float yo = Y[e];
          const float v = yo - alpha * P[e];
          const float yn = v > 0.f ? v : 0.f;
          clip_mine += (v < 0.f) ? 1 : 0;
          Y[e] = yn;
          d = yn - yo;
        }
        P[e] = d;
      }
      // the clipped rows of this update, summed per slot in LDS; read only when the column
      // retires, after many barriers
      if (clip_mine) {
        atomicAdd(&s_clip[slot], clip_mine);
        *s_anyclip = 1;
      }
      __syncthreads();
      // (each thread adds to its own entries of Gr; the next writer of W runs after the
      // barriers of the next statistics reduction, so no barrier is needed after the adds)
      if (*s_anyclip) {
        // grad' = grad + Q d, the second product of Algorithm 2, on the matrix cores
        product(P, W, std::false_type{});
        __syncthreads();
        if (act)
          for (int i = row0; i < n; i += NT / MR_SLOTS)
            Gr[i * MR_SLOTS + slot] += W[i * MR_SLOTS + slot];
      } else if (act) {
        // no slot clipped: d = -alpha gbar in every slot, so Q d = -alpha W with the
        // line-search product W = Q gbar, still intact
        const float alpha = s_alpha[slot];
        for (int i = row0; i < n; i += NT / MR_SLOTS)
          Gr[i * MR_SLOTS + slot] -= alpha * W[i * MR_SLOTS + slot];
      }
    }
    // slot bookkeeping by threads 0..15, each for its own slot (read again only by the same
    // thread in the next decisions)
    if (tid < MR_SLOTS && s_act[tid]) {
      s_it[tid] += 1;
      s_fresh[tid] = 0;
      // rows of Q: the passive rows of the line-search product (the clipped rows are in s_clip)
      const unsigned r = (unsigned)s_rows[tid] + (unsigned)s_cnt[tid];
      if (r < (unsigned)s_rows[tid]) s_rowsh[tid] += 1;
      s_rows[tid] = (int)r;
    }
  }
}


// Register instances (n <= 256, Q in registers in FP32, or as split FP16 parts with SPLIT): the
// update of solve_mrhs_kernel, arranged so that most of it runs in registers.  Thread t works on
// slot c = t % 16 and on the row blocks rb = t / 16 + (NT / 16) j of 8 consecutive rows, which are
// exactly the operand chunks a split writes; its rows of y and of the product operand stay in its
// registers.  The
// state of a slot (column, update count, flags, ||q||) is kept, the same, by every thread of the
// slot: each of them sums the slot's partial statistics and line-search denominator in the same
// order and takes the same decisions, and every wave forms the masks over the 16 slots with one
// ballot (lanes 0..15 of every wave hold slots 0..15).  Threads 0..15 write the outputs.  LDS
// holds the gradient (each thread reads and writes only its own rows of it), the products'
// operands and results and the partial sums, and an update takes three barriers with FP32
// products, four with split ones (one more when a slot clipped).
// Row strides (floats) of the LDS arrays, chosen for their most frequent access.  Product
// results: the epilogue writes rows 4 (l / 16) + e, column l % 16 (lane l), so 20.  Product
// operands: the matrix-core steps read rows 4 ks + l / 16, column l % 16, so 16.  Gradient: the
// update reads rows 8 (t / 16) + e, column t % 16 (thread t), so 18.  Each then hits 64
// distinct banks.
constexpr int MR_PS = 20;
constexpr int MR_PV = 16;
constexpr int MR_PG = 18;
constexpr int MR_REF_BATCH = 4;  // waiting slots that trigger an exact-gradient refresh
constexpr int MR_FEW_PASS = 2;   // FP32 products for at most 4 MR_FEW_PASS slots (updating, or
                                 // waiting for a refresh) take mfma_product_few

template <int TPW, int NT, bool SPLIT>
__global__ __launch_bounds__(NT, NT >= 384 ? 1 : 2) void solve_mrhs_reg_kernel(MrArgs A) {
  constexpr int NW = NT / kWave;
  constexpr int TW = 4 * TPW / NW;            // row tiles of Q per wave
  constexpr int KH = SPLIT ? 2 * TPW : 1;     // k blocks of 32 (split products)
  constexpr int KS = SPLIT ? 1 : 16 * TPW;    // k steps of 4 (FP32 products)
  constexpr int NP = 64 * TPW;                // rows, padded
  constexpr int NB = NT / MR_SLOTS;           // row-block groups
  constexpr int RB = NP / 8;                  // row blocks of 8
  constexpr int JB = (RB + NB - 1) / NB;      // row blocks per thread
  constexpr int S = MR_PS, SV = MR_PV, SG = MR_PG;
  static_assert(TPW > 0 && (4 * TPW) % NW == 0, "row tiles per wave");
  extern __shared__ __attribute__((aligned(16))) float sm[];
  float* P = sm;                                   // [NP][SV] product operand (FP32)
  float* W = P + NP * SV;                          // [NP][S] product result
  float* G = W + NP * S;                           // [NP][SG] gradient
  f16x8* Vh = (f16x8*)(G + NP * SG);               // [RB][16] split operand, hi parts
  f16x8* Vl = Vh + (SPLIT ? RB * MR_SLOTS : 0);    // [RB][16] lo parts
  float* rinv = (float*)(Vl + (SPLIT ? RB * MR_SLOTS : 0));  // [NP] 1 / r per row of Q
  float* red = rinv + (SPLIT ? NP : 0);            // [NW][16][4] statistics partials
  float* red2 = red + NW * MR_SLOTS * 4;           // [NW][16] denominator / ||q||^2 partials
  int* s_newcol = (int*)(red2 + NW * MR_SLOTS);    // [16] next column of a retired slot
  int* s_clip = s_newcol + MR_SLOTS;               // [16] clipped rows so far (rows_read)
  int* s_anyclip = s_clip + MR_SLOTS;              // some slot clipped this update

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid & 15, b = tid >> 4;
  const bool leader = tid < MR_SLOTS;
  const int n = A.n, k = A.k;

  // ---- Q in registers: FP16 hi and lo parts, each row scaled by a power of two (split
  // products), or FP32 (lane l holds Q[16 t + l % 16][4 ks + l / 16], the A operand of step ks)
  f16x8 qh[SPLIT ? TW : 1][KH], ql[SPLIT ? TW : 1][KH];
  float qa[SPLIT ? 1 : TW][KS];
  if constexpr (!SPLIT) {
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) {
      const int m = (wave + NW * tt) * 16 + lr;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kk = 4 * ks + lg;
        qa[tt][ks] = (m < n && kk < n) ? A.Q[(int64_t)m * n + kk] : 0.f;
      }
    }
  } else {
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) {
      const int m = (wave + NW * tt) * 16 + lr;
      float v[KH][8];
      float mx = 0.f;
#pragma unroll
      for (int kh = 0; kh < KH; ++kh)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int kk = 32 * kh + 8 * lg + e;
          v[kh][e] = (m < n && kk < n) ? A.Q[(int64_t)m * n + kk] : 0.f;
          mx = fmaxf(mx, fabsf(v[kh][e]));
        }
      // the row's largest entry: the four lanes l % 16 == lr of the wave hold the whole row
      mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
      mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
      const float r = mr_pow2_scale(mx);
      if (lg == 0) rinv[m] = 1.f / r;
#pragma unroll
      for (int kh = 0; kh < KH; ++kh)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = v[kh][e] * r;
          const _Float16 hx = (_Float16)x;
          qh[tt][kh][e] = hx;
          ql[tt][kh][e] = (_Float16)(x - (float)hx);
        }
    }
  }

  // ---- slot state, the same in every thread of the slot
  int col = blockIdx.x * MR_SLOTS + c;
  col = col < k ? col : -1;
  int it = 0;
  // a warm start needs an exact gradient first, unless it was formed before the launch (G0)
  const bool start_exact = A.Y0 == nullptr || A.G0 != nullptr;
  bool fresh = start_exact, ref = !start_exact && col >= 0, done = false;
  int64_t rows = (A.G0 != nullptr && col >= 0) ? n : 0;
  float qn = 1.f;

  // ---- own rows: blocks blk(j), rows 8 blk(j) + e
  float yv[JB][8], pv[JB][8];
  // k made opaque where the column arrays are addressed, so that the eight row offsets i k are
  // formed at each use instead of being kept in registers through the whole solve
  auto opaque_k = [&]() {
    int kk = k;
    asm volatile("" : "+s"(kk));
    return kk;
  };
  auto blk = [&](int j) { return b + NB * j; };
  auto load_rows = [&]() {
    const int kk = opaque_k();
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = 8 * blk(j) + e;
        float yi = 0.f, gi = 0.f;
        if (blk(j) < RB && col >= 0 && i < n) {
          gi = A.G0 ? A.G0[(int64_t)i * kk + col] : A.q[(int64_t)i * kk + col];
          if (A.Y0) {
            yi = A.Y0[(int64_t)i * kk + col];
            yi = yi > 0.f ? yi : 0.f;
          }
        }
        yv[j][e] = yi;
        if (blk(j) < RB) G[i * SG + c] = gi;
      }
  };
  // a predicate over the 16 slots as a bit mask, the same in every wave
  auto mask16 = [&](bool pred) -> unsigned {
    return (unsigned)(__ballot(lane < MR_SLOTS && pred) & 0xffffull);
  };
  // the slot's sum of one value per thread (a barrier inside; red2 is free at every call)
  auto slot_sum1 = [&](float v) -> float {
    v = add_xor32(add_xor16(v));
    if (lane < MR_SLOTS) red2[wave * MR_SLOTS + lane] = v;
    __syncthreads();
    float a = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) a += red2[w * MR_SLOTS + c];
    return a;
  };
  auto qnorm = [&]() {
    const int kk = opaque_k();
    float a = 0.f;
    if (col >= 0)
#pragma unroll
      for (int j = 0; j < JB; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int i = 8 * blk(j) + e;
          if (blk(j) < RB && i < n) {
            const float qi = A.q[(int64_t)i * kk + col];
            a += qi * qi;
          }
        }
    const float t2 = slot_sum1(a);
    qn = t2 > 0.f ? sqrtf(t2) : 1.f;
  };
  auto write_rows_lds = [&](float* dst, const float (&v)[JB][8]) {
#pragma unroll
    for (int j = 0; j < JB; ++j)
      if (blk(j) < RB)
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[(8 * blk(j) + e) * SV + c] = v[j][e];
  };
  auto split_rows = [&](float sig) {
#pragma unroll
    for (int j = 0; j < JB; ++j)
      if (blk(j) < RB) split_chunk(pv[j], sig, Vh + blk(j) * MR_SLOTS + c, Vl + blk(j) * MR_SLOTS + c);
  };
  auto retire = [&](int st, double r) {  // the leader writes the slot's outputs
    if (leader) {
      A.iters[col] = it;
      A.kkt[col] = st == NNLS_NONFINITE_DEV ? __builtin_nan("") : r;
      A.status[col] = st;
      if (A.rows_read) A.rows_read[col] = rows + s_clip[c];
    }
    done = true;
  };

  if (leader) s_clip[c] = 0;
  if (tid == 0) *s_anyclip = 0;
  load_rows();
  qnorm();  // (its barrier also publishes rinv)

  for (;;) {
    // ---- exact gradient for the slots that ask for it, from the FP32 Q in L2: it decides the
    // stop test, where Q y and q nearly cancel.  A refresh costs about as much as one and a half
    // updates, so requests that confirm a stop are gathered: the product runs once MR_REF_BATCH
    // slots wait, or no slot is left to update, or a new column needs its first gradient (a
    // waiting slot only idles meanwhile; it takes no update).
    const unsigned mwait = mask16(ref && col >= 0 && !done);
    const unsigned mbusy = mask16(col >= 0 && !done && !ref);
    if (mwait && (__builtin_popcount(mwait) >= MR_REF_BATCH || mbusy == 0 ||
                  mask16(ref && col >= 0 && !done && it == 0))) {
      write_rows_lds(P, yv);
      __syncthreads();
      if constexpr (SPLIT) {
        // from the FP32 Q in L2 (four k blocks in flight: the split Q leaves few registers free)
        mfma_product<NT, false, 4, S, SV>(A, P, W, nullptr, nullptr);
      } else {
        const int np4 = (__builtin_popcount(mwait) + 3) / 4;
        if (np4 <= MR_FEW_PASS)
          mfma_product_few<TW, KS, NW, false, S, SV>(qa, P, W, nullptr, nullptr, mwait, np4);
        else
          mfma_product_reg<TW, KS, NW, false, S, SV>(qa, P, W, nullptr, nullptr);
      }
      __syncthreads();
      if (ref && col >= 0 && !done) {
        const int kk = opaque_k();
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int i = 8 * blk(j) + e;
            if (blk(j) < RB && i < n) G[i * SG + c] = W[i * S + c] + A.q[(int64_t)i * kk + col];
          }
        ref = false;
        fresh = true;
        rows += n;
      }
    }

    // ---- passive set, masked gradient, statistics of the own rows, then summed over the slot
    const bool live = col >= 0 && !done;
    float num = 0.f, res = 0.f, cnt = 0.f, bad = 0.f;
    {
      float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f;
#pragma unroll
      for (int j = 0; j < JB; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int i = 8 * blk(j) + e;
          const bool ok = blk(j) < RB && live && i < n;
          const float yi = yv[j][e], gi = blk(j) < RB ? G[i * SG + c] : 0.f;
          const bool pas = ok && ((yi > 0.f) || (gi < 0.f));
          const float pi = pas ? gi : 0.f;
          pv[j][e] = pi;
          t0 += pi * pi;
          const float m = yi < gi ? yi : gi;
          t1 += ok ? m * m : 0.f;
          t2 += pas ? 1.f : 0.f;
          t3 += (ok && (!__builtin_isfinite(yi) || !__builtin_isfinite(gi))) ? 1.f : 0.f;
        }
      t0 = add_xor32(add_xor16(t0));
      t1 = add_xor32(add_xor16(t1));
      t2 = add_xor32(add_xor16(t2));
      t3 = add_xor32(add_xor16(t3));
      if (lane < MR_SLOTS) *(f32x4*)(red + (wave * MR_SLOTS + lane) * 4) = (f32x4){t0, t1, t2, t3};
      // FP32 products: the line-search operand goes to LDS before the statistics barrier, which
      // then also publishes it (a column that will not update has only its own result wasted)
      if constexpr (!SPLIT) write_rows_lds(P, pv);
      __syncthreads();
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const f32x4 v = *(const f32x4*)(red + (w * MR_SLOTS + c) * 4);
        num += v[0];
        res += v[1];
        cnt += v[2];
        bad += v[3];
      }
    }

    // ---- decisions: finish, refresh, or update (a slot waiting for its refresh idles)
    bool act = false;
    double r = 0.0;
    if (live && !ref) {
      r = sqrt((double)res) / (double)qn;
      if (leader && A.trace != nullptr && it < A.trace_len) {
        float* tr = A.trace + ((int64_t)col * A.trace_len + it) * 2;
        tr[0] = (float)r;
        tr[1] = num;
      }
      if (bad > 0.f) {
        retire(NNLS_NONFINITE_DEV, r);
      } else if (cnt == 0.f || r <= A.tol) {
        if (fresh) retire(NNLS_CONVERGED_DEV, r);
        else ref = true;
      } else if (it >= A.max_iter) {
        if (fresh) retire(NNLS_MAXITER_DEV, r);
        else ref = true;
      } else {
        act = true;
      }
    }
    if (mask16(col >= 0 && done)) {
      // retired slots write x = y / s and take the next column from the queue
      if (col >= 0 && done) {
        const int kk = opaque_k();
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int i = 8 * blk(j) + e;
            if (blk(j) < RB && i < n)
              A.X[(int64_t)i * kk + col] = A.s ? (float)((double)yv[j][e] / A.s[i]) : yv[j][e];
          }
        if (leader) {
          const int next = atomicAdd(A.queue, 1);
          s_newcol[c] = next < k ? next : -1;
          s_clip[c] = 0;
        }
      }
      __syncthreads();
      if (col >= 0 && done) {
        col = s_newcol[c];
        it = 0;
        done = false;
        fresh = start_exact;
        ref = !start_exact && col >= 0;
        rows = (A.G0 != nullptr && col >= 0) ? n : 0;
        load_rows();
      }
      qnorm();
      continue;  // evaluate the new columns before any update
    }
    if (!mask16(col >= 0)) break;  // every slot empty: the queue is exhausted
    if (!mask16(act)) continue;    // only exact-gradient refreshes are pending

    // ---- W = Q gbar on the matrix cores, with den_c = gbar_c^T W_c from its epilogue
    if (tid == 0) *s_anyclip = 0;
    const float sg = act ? mr_pow2_scale(sqrtf(num)) : 1.f;  // |gbar_i| <= ||gbar||
    if constexpr (SPLIT) {
      write_rows_lds(P, pv);
      split_rows(sg);
      __syncthreads();
    }
    if constexpr (SPLIT) mfma_product_h3<TW, KH, NW, S, true, SV>(qh, ql, Vh, Vl, rinv, 1.f / sg, W, P, red2);
    else {
      const unsigned ma = mask16(act);
      const int np4 = (__builtin_popcount(ma) + 3) / 4;
      if (np4 <= MR_FEW_PASS) mfma_product_few<TW, KS, NW, true, S, SV>(qa, P, W, P, red2, ma, np4);
      else mfma_product_reg<TW, KS, NW, true, S, SV>(qa, P, W, P, red2);
    }
    __syncthreads();

    // ---- step length, projected update y' = [y - alpha gbar]_+ of the own rows, d = y' - y
    float alpha = 0.f;
    if (act) {
      float den = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) den += red2[w * MR_SLOTS + c];
      if (!(den > 0.f) || !__builtin_isfinite(den)) {
        retire(NNLS_BREAKDOWN_DEV, r);  // the column keeps its current iterate
        act = false;
      } else {
        alpha = num / den;
      }
    }
    int clip_mine = 0;
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = 8 * blk(j) + e;
        float d = 0.f;
        if (act && blk(j) < RB && i < n) {
          const float yo = yv[j][e];
          const float v = yo - alpha * pv[j][e];
          const float yn = v > 0.f ? v : 0.f;
          clip_mine += (v < 0.f) ? 1 : 0;
          yv[j][e] = yn;
          d = yn - yo;
        }
        pv[j][e] = d;
      }
    if (clip_mine) {
      atomicAdd(&s_clip[c], clip_mine);
      *s_anyclip = 1;
    }
    // |y'_i - y_i| <= alpha |gbar_i| <= alpha ||gbar|| (a clipped entry moves less)
    const float sd = act ? mr_pow2_scale(alpha * sqrtf(num)) : 1.f;
    if constexpr (SPLIT) split_rows(sd);
    else write_rows_lds(P, pv);  // (the epilogue's last read of P was before the barrier above)
    __syncthreads();

    // ---- gradient g' = g + Q d, the second product of Algorithm 2; when no slot clipped,
    // d = -alpha gbar in every slot and Q d = -alpha W from the line-search product
    if (*s_anyclip) {
      if constexpr (SPLIT)
        mfma_product_h3<TW, KH, NW, S, false>(qh, ql, Vh, Vl, rinv, 1.f / sd, W, nullptr, nullptr);
      else {
        const unsigned ma = mask16(act);
        const int np4 = (__builtin_popcount(ma) + 3) / 4;
        if (np4 <= MR_FEW_PASS)
          mfma_product_few<TW, KS, NW, false, S, SV>(qa, P, W, nullptr, nullptr, ma, np4);
        else
          mfma_product_reg<TW, KS, NW, false, S, SV>(qa, P, W, nullptr, nullptr);
      }
      __syncthreads();
      if (act)
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int i = 8 * blk(j) + e;
            if (blk(j) < RB && i < n) G[i * SG + c] += W[i * S + c];
          }
    } else if (act) {
#pragma unroll
      for (int j = 0; j < JB; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int i = 8 * blk(j) + e;
          if (blk(j) < RB && i < n) G[i * SG + c] -= alpha * W[i * S + c];
        }
    }
    if (act) {
      it += 1;
      fresh = false;
      rows += (int64_t)cnt;  // the passive rows of the line-search product
    }
  }
}

__global__ void solve_mrhs_queue_init(int* queue, int first_free) {
  if (threadIdx.x == 0) queue[0] = first_free;
}

// ---- host side ------------------------------------------------------------------------------
static int mr_tpw(int64_t n) { return n <= 256 ? (int)((n + 63) / 64) : 0; }
static int mr_np(int64_t n) {
  const int tpw = mr_tpw(n);
  return tpw > 0 ? 64 * tpw : (int)((n + 15) / 16 * 16);
}

// n <= 256: solve_mrhs_reg_kernel (Q in registers); threads per workgroup 512 for four row tiles
// per wave group, 384 for three (6 waves of two tiles, which leaves the registers Q and the own
// rows need), else 256.  n > 256: solve_mrhs_kernel, 256 threads.
static int mr_nt(int64_t n) {
  const int tpw = mr_tpw(n);
  return tpw == 4 ? 512 : (tpw == 3 ? 384 : MR_NT);
}

// Products of the register kernel: FP32 (v_mfma_f32_16x16x4f32) by default, or the split FP16
// form (three v_mfma_f32_16x16x32_f16 per product, each term within 3 2^-22 of the FP32 one)
// with NNLS_MRHS_PRODUCT=split16.
static bool mr_split(int64_t n) {
  if (mr_tpw(n) == 0) return false;
  const char* v = getenv("NNLS_MRHS_PRODUCT");
  return v != nullptr && strcmp(v, "split16") == 0;
}

static size_t mr_lds_bytes(int64_t n, bool split) {
  const size_t np = (size_t)mr_np(n);
  const size_t nw = (size_t)mr_nt(n) / kWave;
  if (mr_tpw(n) > 0)  // solve_mrhs_reg_kernel's layout
    return sizeof(float) * np * (MR_PV + MR_PS + MR_PG) +
           (split ? 2 * sizeof(f16x8) * (np / 8) * MR_SLOTS + sizeof(float) * np : 0) +
           sizeof(float) * nw * MR_SLOTS * 5 + sizeof(int) * 2 * MR_SLOTS + 64;
  return sizeof(float) * 4 * np * MR_SLOTS +
         sizeof(float) * 8 * MR_SLOTS + sizeof(int) * 9 * MR_SLOTS +
         sizeof(float) * nw * MR_SLOTS * 4 + sizeof(int) * 8 + 64;
}

bool solve_mrhs_supported(int64_t n, int64_t k) {
  // (the larger layout, so the answer does not depend on the product form)
  return k >= 2 && n >= 1 && (n % 4) == 0 && mr_lds_bytes(n, true) <= 160 * 1024;
}

size_t solve_mrhs_ws_bytes() { return 256; }

hipError_t launch_solve_mrhs(int64_t n, int64_t k, const float* Q, const float* q,
                             const double* s, double tol, int max_iter, const float* Y0,
                             float* X, int32_t* iters, double* kkt, int32_t* status,
                             int64_t* rows_read, float* trace, int trace_len, void* ws,
                             hipStream_t st) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const bool split = mr_split(n);
  const size_t lds = mr_lds_bytes(n, split);  // the layout of the instance picked below
  const void* kern = nullptr;
#define MR_REG(TPW, NT)                                                    \
  kern = split ? (const void*)solve_mrhs_reg_kernel<TPW, NT, true>        \
               : (const void*)solve_mrhs_reg_kernel<TPW, NT, false>
  switch (mr_tpw(n)) {
    case 1: MR_REG(1, MR_NT); break;
    case 2: MR_REG(2, MR_NT); break;
    case 3: MR_REG(3, 384); break;
    case 4: MR_REG(4, 512); break;
    default: kern = (const void*)solve_mrhs_kernel<MR_NT>; break;
  }
#undef MR_REG
  const int nt = mr_nt(n);
  int per_cu = 1;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int64_t groups = (k + MR_SLOTS - 1) / MR_SLOTS;
  const int64_t resident = (int64_t)cus * per_cu;
  if (groups > resident) groups = resident;
  MrArgs A;
  A.n = (int)n;
  A.np = mr_np(n);
  A.k = (int)k;
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
  A.queue = (int*)ws;
  A.G0 = nullptr;
  // Register kernel, warm start: the start gradients of all columns in one pass, written to X
  // (each column's entries are read when it enters a slot and overwritten only when it
  // retires, by the same workgroup).  Not when X overlaps Y0.
  const size_t nk = (size_t)n * (size_t)k;
  const bool overlap = Y0 != nullptr && (const float*)X < Y0 + nk && Y0 < (const float*)X + nk;
  if (mr_tpw(n) > 0 && Y0 != nullptr && !overlap && A.np <= SG_NP) {
    A.G0 = X;
    hipLaunchKernelGGL(mrhs_start_grad_kernel, dim3((unsigned)((k + MR_SLOTS - 1) / MR_SLOTS)),
                       dim3(MR_NT), 0, st, A, X);
  }
  hipLaunchKernelGGL(solve_mrhs_queue_init, dim3(1), dim3(64), 0, st, A.queue,
                     (int)(groups * MR_SLOTS));
  void* args[] = {&A};
  e = hipLaunchKernel(kern, dim3((unsigned)groups), dim3((unsigned)nt), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace nnls
