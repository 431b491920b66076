// Learned warm start for Algorithm 2: a 256 -> 1024 -> 1024 -> 256 GELU network mapping the
// normalised rescaled right-hand side u = q / ||q|| to one 256-wide head z, read two ways: the
// direction v = ReLU(z) of the start point and the passive-set logit z.  The start itself is
// y0 = c* v with c* the exact line-search step of f along v (the same kind of step Algorithm 2
// takes), so only the direction has to be learned.  Training minimises
//     1/2 ||ReLU(z) - y* / ||y*|| ||^2 + lambda * BCE(z, 1[y* > 0])        (mean over the batch)
// with Adam on FP32 master weights; products run on BF16 copies with FP32 accumulation.
//
// Kernels: one BF16 GEMM on the matrix cores (v_mfma_f32_16x16x32_bf16, 64 x 64 tiles, operands
// transposed as needed while staged into LDS) with fused epilogues (bias + GELU keeping the
// pre-activation, bias, plain FP32, GELU backward); the loss and its gradient; column sums for
// bias gradients; Adam; and the warm-start assembly (line-search scale, and the fallback to y = 0
// when v gives no descent).
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/nnls.h"
#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int ML_IN = 256, ML_H = 1024, ML_OUT = 256;
// parameter layout (elements): W1 [IN, H], b1 [H], W2 [H, H], b2 [H], W3 [H, OUT], b3 [OUT]
constexpr int64_t ML_W1 = 0;
constexpr int64_t ML_B1 = ML_W1 + (int64_t)ML_IN * ML_H;
constexpr int64_t ML_W2 = ML_B1 + ML_H;
constexpr int64_t ML_B2 = ML_W2 + (int64_t)ML_H * ML_H;
constexpr int64_t ML_W3 = ML_B2 + ML_H;
constexpr int64_t ML_B3 = ML_W3 + (int64_t)ML_H * ML_OUT;
constexpr int64_t ML_P = ML_B3 + ML_OUT;
// blob: FP32 master [P], Adam m [P], Adam v [P], BF16 copy [P], input shift [IN], input scale [IN]
constexpr size_t ML_NORM = sizeof(float) * 3 * ML_P + sizeof(uint16_t) * ML_P;
constexpr size_t ML_BLOB = ML_NORM + sizeof(float) * 2 * ML_IN;

typedef uint16_t bf16_t;

__device__ __forceinline__ bf16_t to_bf16(float x) { return (bf16_t)bf16_bits_rne(x); }
__device__ __forceinline__ float from_bf16(bf16_t b) { return bf16_bits_to_f32(b); }

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float cdf = 0.5f * (1.f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

enum { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

struct GemmEpi {
  float* out_f32;        // EPI_F32, EPI_BIAS_F32, EPI_BIAS_GELU (pre-activation; may be
                         // null there when no backward pass follows)
  bf16_t* out_bf16;      // EPI_BIAS_GELU (activation), EPI_GELU_BWD (gradient)
  const float* bias;     // EPI_BIAS_*
  const float* pre;      // EPI_GELU_BWD: pre-activation of the layer
  int64_t ldc;
};

constexpr int MG_BK = 32;
constexpr int MG_LDK = 40;

// C[M, N] = op(A)[M, K] op(B)[K, N], bf16 inputs, FP32 accumulation.
// op(A)(m, k) = TA ? A[k * lda + m] : A[m * lda + k];  op(B)(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n].
// T x T output tiles (T = 64 or 128) on 4 waves of T/2 x T/2 (FT x FT fragments of
// v_mfma_f32_16x16x32_bf16); K in steps of 32, the next step's operands loaded into registers
// while the current step's MFMAs run.  Requires M, N multiples of T and K a multiple of 32
// (checked on the host).
template <bool TA, bool TB, int EPI, int T>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(int M, int N, int K,
                                                       const bf16_t* __restrict__ A, int64_t lda,
                                                       const bf16_t* __restrict__ B, int64_t ldb,
                                                       GemmEpi E) {
  constexpr int FT = T / 32;        // fragments per wave and dimension
  constexpr int LV = T * MG_BK / 8 / 256;  // 16-byte loads per thread and operand per step
  __shared__ __attribute__((aligned(16))) bf16_t sA[T * MG_LDK];
  __shared__ __attribute__((aligned(16))) bf16_t sB[T * MG_LDK];
  const int m0 = blockIdx.x * T, n0 = blockIdx.y * T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (T / 2), wn = (wave & 1) * (T / 2);
  f32x4 acc[FT][FT];
#pragma unroll
  for (int a = 0; a < FT; ++a)
#pragma unroll
    for (int b = 0; b < FT; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

  u32x4 ra[LV], rb[LV];
  // load v of a step: !TA: row m = q / 4 of the tile, k = (q % 4) * 8 .. + 7; TA: k = q / (T/8),
  // m = (q % (T/8)) * 8 .. + 7, with q = tid + 256 v (the same for B with n in place of m)
  auto load = [&](int k0) {
#pragma unroll
    for (int v = 0; v < LV; ++v) {
      const int qd = tid + 256 * v;
      if (!TA) ra[v] = *(const u32x4*)(A + (int64_t)(m0 + (qd >> 2)) * lda + k0 + (qd & 3) * 8);
      else ra[v] = *(const u32x4*)(A + (int64_t)(k0 + qd / (T / 8)) * lda + m0 + (qd % (T / 8)) * 8);
      if (TB) rb[v] = *(const u32x4*)(B + (int64_t)(n0 + (qd >> 2)) * ldb + k0 + (qd & 3) * 8);
      else rb[v] = *(const u32x4*)(B + (int64_t)(k0 + qd / (T / 8)) * ldb + n0 + (qd % (T / 8)) * 8);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int v = 0; v < LV; ++v) {
      const int qd = tid + 256 * v;
      if (!TA) {
        *(u32x4*)&sA[(qd >> 2) * MG_LDK + (qd & 3) * 8] = ra[v];
      } else {
        const int kk = qd / (T / 8), mm = (qd % (T / 8)) * 8;
        const bf16_t* e = (const bf16_t*)&ra[v];
#pragma unroll
        for (int j = 0; j < 8; ++j) sA[(mm + j) * MG_LDK + kk] = e[j];
      }
      if (TB) {
        *(u32x4*)&sB[(qd >> 2) * MG_LDK + (qd & 3) * 8] = rb[v];
      } else {
        const int kk = qd / (T / 8), nn = (qd % (T / 8)) * 8;
        const bf16_t* e = (const bf16_t*)&rb[v];
#pragma unroll
        for (int j = 0; j < 8; ++j) sB[(nn + j) * MG_LDK + kk] = e[j];
      }
    }
  };

  load(0);
  for (int k0 = 0; k0 < K; k0 += MG_BK) {
    store();
    __syncthreads();
    if (k0 + MG_BK < K) load(k0 + MG_BK);  // in flight during the MFMAs below
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 af[FT], bf[FT];
#pragma unroll
    for (int t = 0; t < FT; ++t) {
      af[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&sA[(wm + t * 16 + fr) * MG_LDK + fk]);
      bf[t] = __builtin_bit_cast(bf16x8, *(const u32x4*)&sB[(wn + t * 16 + fr) * MG_LDK + fk]);
    }
#pragma unroll
    for (int a = 0; a < FT; ++a)
#pragma unroll
      for (int b = 0; b < FT; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bf[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  const int oc = lane & 15, orow = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < FT; ++a)
#pragma unroll
    for (int b = 0; b < FT; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + wm + a * 16 + orow + e;
        const int64_t n = n0 + wn + b * 16 + oc;
        const float v = acc[a][b][e];
        const int64_t o = m * E.ldc + n;
        if (EPI == EPI_F32) {
          E.out_f32[o] = v;
        } else if (EPI == EPI_BIAS_F32) {
          E.out_f32[o] = v + E.bias[n];
        } else if (EPI == EPI_BIAS_GELU) {
          const float pre = v + E.bias[n];
          if (E.out_f32) E.out_f32[o] = pre;  // kept for the backward pass only
          E.out_bf16[o] = to_bf16(gelu(pre));
        } else {
          E.out_bf16[o] = to_bf16(v * gelu_grad(E.pre[o]));
        }
      }
}

// 128 x 128 tiles where M and N allow it and there are at least 512 of them (a wave then runs
// 16 MFMAs per K step instead of 4), else 64 x 64 (the small products of training would leave
// most of the GPU idle with the larger tiles).
template <bool TA, bool TB, int EPI>
static void gemm(int M, int N, int K, const bf16_t* A, int64_t lda, const bf16_t* B, int64_t ldb,
                 GemmEpi E, hipStream_t st) {
  if (M % 128 == 0 && N % 128 == 0 && (int64_t)(M / 128) * (N / 128) >= 512) {
    dim3 grid((unsigned)(M / 128), (unsigned)(N / 128));
    hipLaunchKernelGGL((mlp_gemm_kernel<TA, TB, EPI, 128>), grid, dim3(256), 0, st, M, N, K, A,
                       lda, B, ldb, E);
  } else {
    dim3 grid((unsigned)(M / 64), (unsigned)(N / 64));
    hipLaunchKernelGGL((mlp_gemm_kernel<TA, TB, EPI, 64>), grid, dim3(256), 0, st, M, N, K, A,
                       lda, B, ldb, E);
  }
}

// X[b, j] = bf16((u[b, j] - shift[j]) * scale[j]): the input standardisation, applied in FP32
// before the BF16 rounding (the informative part of u can be a small fraction of its size).
__global__ void input_kernel(int64_t count, const float* __restrict__ u,
                             const float* __restrict__ shift, const float* __restrict__ scale,
                             bf16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) {
    const int j = (int)(i & (ML_IN - 1));
    y[i] = to_bf16((u[i] - shift[j]) * scale[j]);
  }
}

// Input statistics over `count` rows of U [count, 256], first pass: block b sums rows
// b, b + FI_CHUNKS, ... of (u - u[0]) and its square in FP64 (thread j = feature j, so each row
// is one coalesced read).  Shifting by the first row keeps the variance free of cancellation.
constexpr int FI_CHUNKS = 256;
__global__ __launch_bounds__(256) void fit_input_partial_kernel(int64_t count,
                                                                const float* __restrict__ U,
                                                                double* __restrict__ part) {
  const int j = threadIdx.x;
  const double ref = U[j];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = blockIdx.x; r < count; r += FI_CHUNKS) {
    const double d = (double)U[r * ML_IN + j] - ref;
    s1 += d;
    s2 += d * d;
  }
  part[(int64_t)blockIdx.x * 2 * ML_IN + j] = s1;
  part[(int64_t)blockIdx.x * 2 * ML_IN + ML_IN + j] = s2;
}

// Second pass: shift = mean, scale = 1 / standard deviation (population), 1 where it is 0.
__global__ __launch_bounds__(256) void fit_input_final_kernel(int64_t count,
                                                              const float* __restrict__ U,
                                                              const double* __restrict__ part,
                                                              float* __restrict__ shift,
                                                              float* __restrict__ scale) {
  const int j = threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int c = 0; c < FI_CHUNKS; ++c) {
    s1 += part[(int64_t)c * 2 * ML_IN + j];
    s2 += part[(int64_t)c * 2 * ML_IN + ML_IN + j];
  }
  const double m = s1 / (double)count;
  double var = s2 / (double)count - m * m;
  var = var > 0.0 ? var : 0.0;
  shift[j] = (float)((double)U[j] + m);
  scale[j] = var > 0.0 ? (float)(1.0 / sqrt(var)) : 1.f;
}

// Loss and its gradient w.r.t. z (scaled by 1 / batch), per row block; loss partial per block.
__global__ __launch_bounds__(256) void mlp_loss_kernel(int64_t batch, const float* __restrict__ Z,
                                                       const float* __restrict__ T, float lambda,
                                                       bf16_t* __restrict__ dZ,
                                                       float* __restrict__ loss_part) {
  __shared__ float red[4];
  const int64_t r = blockIdx.x;  // one row per block, 256 outputs per row
  const int j = threadIdx.x;
  const int64_t o = r * ML_OUT + j;
  const float z = Z[o], t = T[o];
  const float relu = z > 0.f ? z : 0.f;
  const float lab = t > 0.f ? 1.f : 0.f;
  const float diff = relu - t;
  // BCE with logits, stable form: max(z,0) - z*lab + log(1 + exp(-|z|))
  const float bce = relu - z * lab + log1pf(expf(-fabsf(z)));
  const float sig = 1.f / (1.f + expf(-z));
  const float g = (diff * (z > 0.f ? 1.f : 0.f) + lambda * (sig - lab)) / (float)batch;
  dZ[o] = to_bf16(g);
  float l = 0.5f * diff * diff + lambda * bce;
  l = block_sum<float, 256>(l, red);
  if (j == 0) loss_part[r] = l / (float)batch;
}

// Bias gradients out[j] = sum_r in[r, j] of a BF16 [rows, cols] matrix, in two stages so that
// the sum over the batch is spread over many workgroups: stage 1, block (256 columns, chunk c of
// the rows) sums its rows per column into part[c][j]; stage 2 adds the chunk partials of each
// column in chunk order.  Chunks of max(32, ceil(rows / 64)) rows keep at most 64 partials.
constexpr int64_t CS_MAX_CHUNKS = 64;
static int64_t colsum_chunk_rows(int64_t rows) {
  const int64_t r = (rows + CS_MAX_CHUNKS - 1) / CS_MAX_CHUNKS;
  return r > 32 ? r : 32;
}

__global__ __launch_bounds__(256) void colsum_partial_kernel(int64_t rows, int64_t cols,
                                                             int64_t chunk_rows,
                                                             const bf16_t* __restrict__ in,
                                                             float* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  const int64_t r0 = (int64_t)blockIdx.y * chunk_rows;
  const int64_t r1 = r0 + chunk_rows < rows ? r0 + chunk_rows : rows;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  int64_t r = r0;
  for (; r + 7 < r1; r += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = from_bf16(in[(r + u) * cols + j]);
    a0 += v[0] + v[4];
    a1 += v[1] + v[5];
    a2 += v[2] + v[6];
    a3 += v[3] + v[7];
  }
  for (; r < r1; ++r) a0 += from_bf16(in[r * cols + j]);
  part[(int64_t)blockIdx.y * cols + j] = (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(256) void colsum_finish_kernel(int64_t chunks, int64_t cols,
                                                            const float* __restrict__ part,
                                                            float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float a = 0.f;
  for (int64_t c = 0; c < chunks; ++c) a += part[c * cols + j];
  out[j] = a;
}

static void colsum(int64_t rows, int64_t cols, const bf16_t* in, float* part, float* out,
                   hipStream_t st) {
  const int64_t cr = colsum_chunk_rows(rows);
  const int64_t chunks = (rows + cr - 1) / cr;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((unsigned)((cols + 255) / 256), (unsigned)chunks),
                     dim3(256), 0, st, rows, cols, cr, in, part);
  hipLaunchKernelGGL(colsum_finish_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st,
                     chunks, cols, (const float*)part, out);
}

__global__ void sum_kernel(int64_t count, const float* __restrict__ in, float* __restrict__ out) {
  __shared__ float red[4];
  float a = 0.f;
  for (int64_t i = threadIdx.x; i < count; i += 256) a += in[i];
  a = block_sum<float, 256>(a, red);
  if (threadIdx.x == 0) out[0] = a;
}

// Adam (bias-corrected) on the FP32 master weights, then the BF16 copy.
__global__ void adam_kernel(int64_t count, float* __restrict__ w, float* __restrict__ m,
                            float* __restrict__ v, bf16_t* __restrict__ wb,
                            const float* __restrict__ g, float lr, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = to_bf16(wi);
}

__global__ void reset_state_kernel(int64_t count, const float* __restrict__ w,
                                   float* __restrict__ m, float* __restrict__ v,
                                   bf16_t* __restrict__ wb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  m[i] = 0.f;
  v[i] = 0.f;
  wb[i] = to_bf16(w[i]);
}

// ---- workspace layout ------------------------------------------------------------------------
struct MlpWs {
  bf16_t *X, *A1, *A2, *dZ, *dH2, *dH1, *WT;
  float *H1, *H2, *Z, *grad, *loss_part, *loss, *colpart;
};

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

static MlpWs mlp_layout(void* ws, int64_t batch, bool train, size_t* total) {
  MlpWs W{};
  char* p = (char*)ws;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void* r = p ? (void*)(p + off) : nullptr;
    off += al(bytes);
    return r;
  };
  W.X = (bf16_t*)take(2 * batch * ML_IN);
  W.H1 = (float*)take(4 * batch * ML_H);
  W.A1 = (bf16_t*)take(2 * batch * ML_H);
  W.H2 = (float*)take(4 * batch * ML_H);
  W.A2 = (bf16_t*)take(2 * batch * ML_H);
  W.Z = (float*)take(4 * batch * ML_OUT);
  W.WT = (bf16_t*)take(2 * ML_P);  // the BF16 weights transposed, for the forward products
  if (train) {
    W.dZ = (bf16_t*)take(2 * batch * ML_OUT);
    W.dH2 = (bf16_t*)take(2 * batch * ML_H);
    W.dH1 = (bf16_t*)take(2 * batch * ML_H);
    W.grad = (float*)take(4 * ML_P);
    W.loss_part = (float*)take(4 * batch);
    W.loss = (float*)take(4);
    W.colpart = (float*)take(4 * CS_MAX_CHUNKS * ML_H);
  }
  if (total) *total = off;
  return W;
}

size_t mlp_ws_bytes(int64_t batch, bool train) {
  size_t t = 0;
  mlp_layout(nullptr, batch, train, &t);
  return t;
}

// dst[c, r] = src[r, c] for a bf16 [rows, cols] matrix (rows, cols multiples of 32), through a
// 32 x 33 LDS tile.
__global__ __launch_bounds__(256) void bf16_transpose_kernel(int64_t rows, int64_t cols,
                                                             const bf16_t* __restrict__ src,
                                                             bf16_t* __restrict__ dst) {
  __shared__ bf16_t t[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += 8) t[y][threadIdx.x] = src[(r0 + y) * cols + c0 + threadIdx.x];
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += 8) dst[(c0 + y) * rows + r0 + threadIdx.x] = t[threadIdx.x][y];
}

static const bf16_t* wcopy(const void* blob) {
  return (const bf16_t*)((const char*)blob + sizeof(float) * 3 * ML_P);
}
static const float* norm_shift(const void* blob) {
  return (const float*)((const char*)blob + ML_NORM);
}
static const float* norm_scale(const void* blob) { return norm_shift(blob) + ML_IN; }

// forward pass; leaves A1, A2 and Z in the workspace, and the pre-activations H1, H2 when a
// backward pass follows (keep_pre).  The products read each weight matrix as W^T (rows of W^T
// are k-contiguous, the layout the staging copies into LDS as is), from a transposed copy made
// first.
static void forward(int64_t batch, const void* blob, const float* u, const MlpWs& W,
                    hipStream_t st, bool keep_pre) {
  const bf16_t* Wb = wcopy(blob);
  const float* master = (const float*)blob;
  const int M = (int)batch;
  struct {
    int64_t off, rows, cols;
  } const mats[3] = {{ML_W1, ML_IN, ML_H}, {ML_W2, ML_H, ML_H}, {ML_W3, ML_H, ML_OUT}};
  for (const auto& m : mats)
    hipLaunchKernelGGL(bf16_transpose_kernel, dim3((unsigned)(m.cols / 32), (unsigned)(m.rows / 32)),
                       dim3(32, 8), 0, st, m.rows, m.cols, Wb + m.off, W.WT + m.off);
  hipLaunchKernelGGL(input_kernel, dim3((unsigned)((batch * ML_IN + 255) / 256)), dim3(256), 0,
                     st, batch * ML_IN, u, norm_shift(blob), norm_scale(blob), W.X);
  GemmEpi e1{keep_pre ? W.H1 : nullptr, W.A1, master + ML_B1, nullptr, ML_H};
  gemm<false, true, EPI_BIAS_GELU>(M, ML_H, ML_IN, W.X, ML_IN, W.WT + ML_W1, ML_IN, e1, st);
  GemmEpi e2{keep_pre ? W.H2 : nullptr, W.A2, master + ML_B2, nullptr, ML_H};
  gemm<false, true, EPI_BIAS_GELU>(M, ML_H, ML_H, W.A1, ML_H, W.WT + ML_W2, ML_H, e2, st);
  GemmEpi e3{W.Z, nullptr, master + ML_B3, nullptr, ML_OUT};
  gemm<false, true, EPI_BIAS_F32>(M, ML_OUT, ML_H, W.A2, ML_H, W.WT + ML_W3, ML_H, e3, st);
}

// loss, then gradients of every parameter into W.grad (same layout as the parameters)
static void backward(int64_t batch, const void* blob, const float* target, float lambda,
                     const MlpWs& W, hipStream_t st) {
  const bf16_t* Wb = wcopy(blob);
  const int M = (int)batch;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3((unsigned)batch), dim3(256), 0, st, batch, W.Z, target,
                     lambda, W.dZ, W.loss_part);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, batch, (const float*)W.loss_part,
                     W.loss);
  // layer 3: dW3 = A2^T dZ, db3 = colsum dZ, dA2 = dZ W3^T -> dH2 = dA2 * gelu'(H2)
  GemmEpi g3{W.grad + ML_W3, nullptr, nullptr, nullptr, ML_OUT};
  gemm<true, false, EPI_F32>(ML_H, ML_OUT, M, W.A2, ML_H, W.dZ, ML_OUT, g3, st);
  colsum(batch, ML_OUT, W.dZ, W.colpart, W.grad + ML_B3, st);
  GemmEpi d2{nullptr, W.dH2, nullptr, W.H2, ML_H};
  gemm<false, true, EPI_GELU_BWD>(M, ML_H, ML_OUT, W.dZ, ML_OUT, Wb + ML_W3, ML_OUT, d2, st);
  // layer 2
  GemmEpi g2{W.grad + ML_W2, nullptr, nullptr, nullptr, ML_H};
  gemm<true, false, EPI_F32>(ML_H, ML_H, M, W.A1, ML_H, W.dH2, ML_H, g2, st);
  colsum(batch, ML_H, W.dH2, W.colpart, W.grad + ML_B2, st);
  GemmEpi d1{nullptr, W.dH1, nullptr, W.H1, ML_H};
  gemm<false, true, EPI_GELU_BWD>(M, ML_H, ML_H, W.dH2, ML_H, Wb + ML_W2, ML_H, d1, st);
  // layer 1
  GemmEpi g1{W.grad + ML_W1, nullptr, nullptr, nullptr, ML_H};
  gemm<true, false, EPI_F32>(ML_IN, ML_H, M, W.X, ML_IN, W.dH1, ML_H, g1, st);
  colsum(batch, ML_H, W.dH1, W.colpart, W.grad + ML_B1, st);
}

// ---- warm start ------------------------------------------------------------------------------
constexpr int WS_C = 16;  // columns per block: q and Y0 rows are read and written 16 floats wide

// For columns c0..c0+15 of q [n = 256, k]: u_c = q_c / ||q_c|| as row c of U [rows, n]
// (rows >= k: rows c >= k, the batch padding, are zero).  With Y [n, k] given, also the unit
// target T[c, :] = Y[:, c] / ||Y_c|| (zero for a zero column).  Thread i owns row i of q and Y.
__global__ __launch_bounds__(256) void ws_normalise_kernel(int64_t k, int64_t rows,
                                                           const float* __restrict__ q,
                                                           const float* __restrict__ Y,
                                                           float* __restrict__ U,
                                                           float* __restrict__ T) {
  __shared__ float red[2][WS_C][4];
  const int i = threadIdx.x, lane = i & 63, wave = i >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * WS_C;
  float v[WS_C], w[WS_C];
#pragma unroll
  for (int c = 0; c < WS_C; ++c) {
    const bool in = c0 + c < k;
    v[c] = in ? q[(int64_t)i * k + c0 + c] : 0.f;
    w[c] = (in && Y) ? Y[(int64_t)i * k + c0 + c] : 0.f;
  }
#pragma unroll
  for (int c = 0; c < WS_C; ++c) {
    const float t0 = wave_sum(v[c] * v[c]);
    const float t1 = wave_sum(w[c] * w[c]);
    if (lane == 0) {
      red[0][c][wave] = t0;
      red[1][c][wave] = t1;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < WS_C; ++c) {
    if (c0 + c >= rows) break;
    const float a = (red[0][c][0] + red[0][c][1]) + (red[0][c][2] + red[0][c][3]);
    U[(c0 + c) * ML_IN + i] = v[c] / (a > 0.f ? sqrtf(a) : 1.f);
    if (Y) {
      const float b = (red[1][c][0] + red[1][c][1]) + (red[1][c][2] + red[1][c][3]);
      T[(c0 + c) * ML_IN + i] = w[c] / (b > 0.f ? sqrtf(b) : 1.f);
    }
  }
}

// Columns c0..c0+15: direction v_c = ReLU(Z[c, :]); then a = v^T Q v and b = q_c^T v with Q read by
// columns (Q is symmetric, so thread i accumulates (Q v)_i from coalesced rows of Q, each row
// reused for the 16 columns).  The start is the exact minimiser of f along v,
//     y0 = c* v,  c* = -b / a,  f(y0) = -b^2 / (2 a) < 0 = f(0),
// taken only when b < 0 and a > 0 with c* finite; otherwise (v = 0, v an ascent direction, NaN
// or inf) the column falls back to the cold start y0 = 0.
__global__ __launch_bounds__(256) void ws_assemble_kernel(int64_t k, const float* __restrict__ Q,
                                                          const float* __restrict__ q,
                                                          const float* __restrict__ Z,
                                                          float* __restrict__ Y0,
                                                          int32_t* __restrict__ fell_back) {
  __shared__ float vs[WS_C][ML_IN];
  __shared__ float red[2][WS_C][4];
  const int i = threadIdx.x, lane = i & 63, wave = i >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * WS_C;
  const int cols = (int)(k - c0 < WS_C ? k - c0 : WS_C);
#pragma unroll
  for (int c = 0; c < WS_C; ++c) {
    float v = 0.f;
    if (c < cols) {
      const float z = Z[(c0 + c) * ML_IN + i];
      v = z > 0.f ? z : 0.f;
      if (z != z) v = z;  // keep a NaN prediction visible to the checks
    }
    vs[c][i] = v;
  }
  __syncthreads();
  float qv[WS_C];
#pragma unroll
  for (int c = 0; c < WS_C; ++c) qv[c] = 0.f;
  for (int j = 0; j < ML_IN; ++j) {
    const float qji = Q[j * ML_IN + i];
#pragma unroll
    for (int c = 0; c < WS_C; ++c) qv[c] += qji * vs[c][j];
  }
#pragma unroll
  for (int c = 0; c < WS_C; ++c) {
    const float vi = vs[c][i];
    const float qi = c < cols ? q[(int64_t)i * k + c0 + c] : 0.f;
    const float ta = wave_sum(vi * qv[c]);
    const float tb = wave_sum(vi * qi);
    if (lane == 0) {
      red[0][c][wave] = ta;
      red[1][c][wave] = tb;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < WS_C; ++c) {
    if (c >= cols) continue;
    const float a = (red[0][c][0] + red[0][c][1]) + (red[0][c][2] + red[0][c][3]);
    const float b = (red[1][c][0] + red[1][c][1]) + (red[1][c][2] + red[1][c][3]);
    const float cs = -b / a;
    const bool take = b < 0.f && a > 0.f && is_finite_val(cs) && is_finite_val(a);
    Y0[(int64_t)i * k + c0 + c] = take ? cs * vs[c][i] : 0.f;
    if (i == 0) fell_back[c0 + c] = take ? 0 : 1;
  }
}

// ---- checkpoints: 64-byte little-endian header, then the blob as it lies in device memory ----
struct CkptHeader {
  char magic[8];       // "NNLSCKP1"
  uint32_t version;    // 1
  uint32_t widths[3];  // ML_IN, ML_H, ML_OUT
  int64_t params;      // ML_P
  uint64_t bytes;      // ML_BLOB
  int64_t step;        // Adam steps taken
  uint64_t hash;       // FNV-1a 64 of the blob bytes
  uint64_t reserved;   // 0
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");
constexpr char kCkptMagic[8] = {'N', 'N', 'L', 'S', 'C', 'K', 'P', '1'};

uint64_t fnv1a64(const unsigned char* p, size_t n) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

}  // namespace nnls

// ---- C ABI -------------------------------------------------------------------------------------
extern "C" {

int nnls_mlp_save(const void* blob, int64_t step, const char* path, void* stream) {
  if (!blob || !path || !*path || step < 0) return NNLS_E_ARG;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return NNLS_E_IO;
  std::vector<unsigned char> host(nnls::ML_BLOB);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(host.data(), blob, nnls::ML_BLOB, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    fclose(f);
    remove(tmp.c_str());
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  nnls::CkptHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, nnls::kCkptMagic, 8);
  h.version = 1;
  h.widths[0] = nnls::ML_IN;
  h.widths[1] = nnls::ML_H;
  h.widths[2] = nnls::ML_OUT;
  h.params = nnls::ML_P;
  h.bytes = nnls::ML_BLOB;
  h.step = step;
  h.hash = nnls::fnv1a64(host.data(), host.size());
  bool ok = fwrite(&h, sizeof(h), 1, f) == 1 && fwrite(host.data(), 1, host.size(), f) == host.size();
  ok = (fflush(f) == 0) && ok;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return NNLS_E_IO;
  }
  return NNLS_OK;
}

int nnls_mlp_load(void* blob, int64_t* step, const char* path, void* stream) {
  if (!blob || !path || !*path) return NNLS_E_ARG;
  FILE* f = fopen(path, "rb");
  if (!f) return NNLS_E_IO;
  nnls::CkptHeader h;
  std::vector<unsigned char> host;
  bool ok = fread(&h, sizeof(h), 1, f) == 1 && memcmp(h.magic, nnls::kCkptMagic, 8) == 0 &&
            h.version == 1 && h.widths[0] == (uint32_t)nnls::ML_IN &&
            h.widths[1] == (uint32_t)nnls::ML_H && h.widths[2] == (uint32_t)nnls::ML_OUT &&
            h.params == nnls::ML_P && h.bytes == (uint64_t)nnls::ML_BLOB && h.step >= 0;
  if (ok) {
    host.resize(nnls::ML_BLOB);
    ok = fread(host.data(), 1, host.size(), f) == host.size() && fgetc(f) == EOF &&
         nnls::fnv1a64(host.data(), host.size()) == h.hash;
  }
  fclose(f);
  if (!ok) return NNLS_E_IO;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(blob, host.data(), nnls::ML_BLOB, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  if (step) *step = h.step;
  return NNLS_OK;
}

int64_t nnls_mlp_param_count(void) { return nnls::ML_P; }

size_t nnls_mlp_blob_bytes(void) { return nnls::ML_BLOB; }

size_t nnls_mlp_workspace_bytes(int64_t batch, int train) {
  if (batch < 1) return 0;
  return nnls::mlp_ws_bytes(batch, train != 0);
}

static int mlp_check_batch(int64_t batch) {
  return (batch >= 64 && batch % 64 == 0 && batch <= (1 << 24)) ? NNLS_OK : NNLS_E_ARG;
}

int nnls_mlp_reset_state(void* blob, void* stream) {
  if (!blob) return NNLS_E_ARG;
  float* w = (float*)blob;
  hipLaunchKernelGGL(nnls::reset_state_kernel, dim3((unsigned)((nnls::ML_P + 255) / 256)),
                     dim3(256), 0, (hipStream_t)stream, nnls::ML_P, (const float*)w,
                     w + nnls::ML_P, w + 2 * nnls::ML_P,
                     (nnls::bf16_t*)(w + 3 * nnls::ML_P));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

size_t nnls_mlp_fit_input_workspace_bytes(void) {
  return sizeof(double) * 2 * nnls::ML_IN * nnls::FI_CHUNKS;
}

int nnls_mlp_fit_input(int64_t count, void* blob, const float* U, void* ws, size_t ws_bytes,
                       void* stream) {
  if (count < 1 || !blob || !U) return NNLS_E_ARG;
  if (!ws || ws_bytes < nnls_mlp_fit_input_workspace_bytes()) return NNLS_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  float* shift = (float*)((char*)blob + nnls::ML_NORM);
  hipLaunchKernelGGL(nnls::fit_input_partial_kernel, dim3(nnls::FI_CHUNKS), dim3(256), 0, st,
                     count, U, (double*)ws);
  hipLaunchKernelGGL(nnls::fit_input_final_kernel, dim3(1), dim3(256), 0, st, count, U,
                     (const double*)ws, shift, shift + nnls::ML_IN);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

int nnls_mlp_forward(int64_t batch, const void* blob, const float* u, float* z, void* ws,
                     size_t ws_bytes, void* stream) {
  if (mlp_check_batch(batch) != NNLS_OK || !blob || !u || !z) return NNLS_E_ARG;
  size_t need = 0;
  nnls::mlp_layout(nullptr, batch, false, &need);
  if (!ws || ws_bytes < need) return NNLS_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  nnls::MlpWs W = nnls::mlp_layout(ws, batch, false, nullptr);
  nnls::forward(batch, blob, u, W, st, false);
  hipError_t e = hipMemcpyAsync(z, W.Z, sizeof(float) * batch * nnls::ML_OUT,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

int nnls_mlp_gradients(int64_t batch, const void* blob, const float* u, const float* target,
                       float lambda, float* grad_out, float* loss_out, void* ws, size_t ws_bytes,
                       void* stream) {
  if (mlp_check_batch(batch) != NNLS_OK || !blob || !u || !target) return NNLS_E_ARG;
  size_t need = 0;
  nnls::mlp_layout(nullptr, batch, true, &need);
  if (!ws || ws_bytes < need) return NNLS_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  nnls::MlpWs W = nnls::mlp_layout(ws, batch, true, nullptr);
  nnls::forward(batch, blob, u, W, st, true);
  nnls::backward(batch, blob, target, lambda, W, st);
  hipError_t e = hipSuccess;
  if (grad_out)
    e = hipMemcpyAsync(grad_out, W.grad, sizeof(float) * nnls::ML_P, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && loss_out)
    e = hipMemcpyAsync(loss_out, W.loss, sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

int nnls_mlp_train_step(int64_t batch, void* blob, const float* u, const float* target,
                        float lr, int64_t step, float lambda, float* loss_out, void* ws,
                        size_t ws_bytes, void* stream) {
  if (step < 1 || !(lr > 0.f)) return NNLS_E_ARG;
  int rc = nnls_mlp_gradients(batch, blob, u, target, lambda, nullptr, loss_out, ws, ws_bytes,
                              stream);
  if (rc != NNLS_OK) return rc;
  nnls::MlpWs W = nnls::mlp_layout(ws, batch, true, nullptr);
  float* w = (float*)blob;
  const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(nnls::adam_kernel, dim3((unsigned)((nnls::ML_P + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, nnls::ML_P, w, w + nnls::ML_P, w + 2 * nnls::ML_P,
                     (nnls::bf16_t*)(w + 3 * nnls::ML_P), (const float*)W.grad, lr, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

int nnls_mlp_inputs(int64_t n, int64_t k, const float* q, const float* Y, float* U, float* T,
                    void* stream) {
  if (n != nnls::ML_IN) return n < 1 ? NNLS_E_ARG : NNLS_E_UNSUPPORTED;
  if (k < 1 || k > (int64_t(1) << 30) || !q || !U || (Y && !T)) return NNLS_E_ARG;
  hipLaunchKernelGGL(nnls::ws_normalise_kernel, dim3((unsigned)((k + nnls::WS_C - 1) / nnls::WS_C)),
                     dim3(256), 0, (hipStream_t)stream, k, k, q, Y, U, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

size_t nnls_warm_start_workspace_bytes(int64_t n, int64_t k) {
  if (n != nnls::ML_IN || k < 1 || k > (int64_t(1) << 24)) return 0;
  const int64_t kb = (k + 63) / 64 * 64;
  return nnls::mlp_ws_bytes(kb, false) + nnls::al(sizeof(float) * kb * n);
}

int nnls_warm_start(int64_t n, int64_t k, const float* Q, const float* q, const void* blob,
                    float* Y0, int32_t* fell_back, void* ws, size_t ws_bytes, void* stream) {
  if (n != nnls::ML_IN) return n < 1 ? NNLS_E_ARG : NNLS_E_UNSUPPORTED;
  if (k < 1 || k > (int64_t(1) << 24) || !Q || !q || !blob || !Y0 || !fell_back) return NNLS_E_ARG;
  const size_t need = nnls_warm_start_workspace_bytes(n, k);
  if (!ws || ws_bytes < need) return NNLS_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const int64_t kb = (k + 63) / 64 * 64;
  char* p = (char*)ws;
  nnls::MlpWs W = nnls::mlp_layout(p, kb, false, nullptr);
  float* U = (float*)(p + nnls::mlp_ws_bytes(kb, false));
  hipLaunchKernelGGL(nnls::ws_normalise_kernel, dim3((unsigned)(kb / nnls::WS_C)), dim3(256), 0,
                     st, k, kb, q, (const float*)nullptr, U, (float*)nullptr);
  nnls::forward(kb, blob, U, W, st, false);
  hipLaunchKernelGGL(nnls::ws_assemble_kernel, dim3((unsigned)((k + nnls::WS_C - 1) / nnls::WS_C)),
                     dim3(256), 0, st, k, Q, q, (const float*)W.Z, Y0, fell_back);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    nnls::record_hip_error(e);
    return NNLS_E_HIP;
  }
  return NNLS_OK;
}

}  // extern "C"
