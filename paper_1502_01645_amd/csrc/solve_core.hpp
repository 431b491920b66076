// Device code of Algorithm 2 for one right-hand side handled by one workgroup: shared by the
// per-column solver and the uneven-batch solver.
//
// The workgroup owns one column: y, the gradient and Q*gbar live in caller-provided global
// vectors, the masked gradient and the compacted passive / clipped index lists live in LDS.
// Because Q is symmetric, the product Q * gbar only needs the rows of Q in the passive set
// (each a contiguous row), and the incremental gradient reuses it:
//     grad' = grad + Q (y' - y) = grad - alpha * (Q gbar) + Q[:, C] delta_C,
// where C is the set of entries the projection clipped and delta = (y' - y) + alpha * gbar is
// nonzero only there.  The products over a list of rows are list_product below.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int SW_NT = 256;   // threads of the per-column solver's workgroup
constexpr int LP_VC = 4;     // entries per lane in a chunk of list_product
constexpr int LP_CH = 64 * LP_VC;

template <typename T>
struct SolveCol {
  int64_t n;
  const T* Q;      // [n, n], row stride n
  const T* q;      // column entries q[i * qs]
  int64_t qs;
  const T* y0;     // start entries y0[i * qs] or nullptr
  T* y;            // workspace [n]
  T* g;            // workspace [n]
  T* w;            // workspace [n]: Q gbar of the current pass
  T* x;            // output entries x[i * qs]
  const double* s; // scales or nullptr
  float* trace;    // [trace_len][2] per-update record of this column, or nullptr
  int trace_len;
};

// For every i < n: emit(i, sum over m < cnt of val[m] * Q[idx[m] * n + i]).  Q is symmetric, so
// the list's rows of Q stand for its columns and each is read as a contiguous row.  The entries
// go in chunks of LP_CH; in a chunk, a row is read by one wave (lane l takes entries l + 64 v),
// the waves split the list (wave w takes m = w, w + NW, ..., four rows in flight, so a lane has
// 4 LP_VC loads outstanding), and each wave leaves its partial sums in LDS part[NW][LP_CH].
// The partials are added in wave order: the result does not depend on timing.  emit runs in
// the thread that owns entry i of the chunk (i = c0 + tid + NT u); every thread calls this.
template <typename T, int NT, typename Emit>
__device__ __forceinline__ void list_product(const T* __restrict__ Q, int64_t n,
                                             const int* __restrict__ idx,
                                             const T* __restrict__ val, int cnt, T* part,
                                             Emit emit) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int64_t c0 = 0; c0 < n; c0 += LP_CH) {
    const int64_t rem = n - c0;
    T acc[LP_VC];
#pragma unroll
    for (int v = 0; v < LP_VC; ++v) acc[v] = (T)0;
    int m = wave;
    for (; m + 3 * NW < cnt; m += 4 * NW) {
      T a[4], x[4][LP_VC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T* row = Q + (int64_t)idx[m + u * NW] * n + c0;
        a[u] = val[m + u * NW];
#pragma unroll
        for (int v = 0; v < LP_VC; ++v) {
          const int e = lane + kWave * v;
          x[u][v] = e < rem ? row[e] : (T)0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < LP_VC; ++v) acc[v] += a[u] * x[u][v];
    }
    for (; m < cnt; m += NW) {
      const T* row = Q + (int64_t)idx[m] * n + c0;
      const T a = val[m];
#pragma unroll
      for (int v = 0; v < LP_VC; ++v) {
        const int e = lane + kWave * v;
        acc[v] += a * (e < rem ? row[e] : (T)0);
      }
    }
#pragma unroll
    for (int v = 0; v < LP_VC; ++v) part[wave * LP_CH + lane + kWave * v] = acc[v];
    __syncthreads();
    for (int e = threadIdx.x; e < LP_CH && e < rem; e += NT) {
      T sum = (T)0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += part[w * LP_CH + e];
      emit(c0 + e, sum);
    }
    __syncthreads();
  }
}

// Algorithm 2 on one column by a workgroup of NT threads.  LDS: the passive list (lds_val,
// lds_idx) and the clipped / positive list (lds_val2, lds_idx2) of n entries each, the partial
// sums of list_product (part, NT / 64 x LP_CH), and block-reduction scratch (NT / 64 each).
template <typename T, int NT>
__device__ void solve_column(const SolveCol<T>& P, double tol, int max_iter, int32_t* iters_out,
                             double* kkt_out, int32_t* status_out, int64_t* rows_out,
                             T* lds_val, int* lds_idx,
                             T* lds_val2, int* lds_idx2, T* part, T* redT, int* redI) {
  const int tid = threadIdx.x;
  const int64_t n = P.n;
  const T* __restrict__ Q = P.Q;
  T* __restrict__ y = P.y;
  T* __restrict__ g = P.g;

  // ||q|| for the relative residual; start point.
  T qq = 0;
  int nonfinite = 0;
  for (int64_t i = tid; i < n; i += NT) {
    const T qi = P.q[i * P.qs];
    qq += qi * qi;
    T yi = 0;
    if (P.y0) {
      yi = P.y0[i * P.qs];
      yi = yi > (T)0 ? yi : (T)0;
    }
    nonfinite |= !is_finite_val(qi) || !is_finite_val(yi);
    y[i] = yi;
    g[i] = qi;
  }
  qq = block_sum<T, NT>(qq, redT);
  const T qnorm = sqrt(qq);
  const T scale = qnorm > (T)0 ? qnorm : (T)1;
  __syncthreads();

  int64_t rows = 0;  // rows of Q read by the products
  // Recompute grad = Q y + q exactly over the rows with y_j > 0.
  auto refresh_gradient = [&]() {
    int cnt = 0;
    for (int64_t i = tid; i < n; i += NT) cnt += (y[i] > (T)0);
    int total;
    int off = block_exclusive_scan<NT>(cnt, redI, total);
    for (int64_t i = tid; i < n; i += NT) {
      const T yi = y[i];
      if (yi > (T)0) {
        lds_idx2[off] = (int)i;
        lds_val2[off] = yi;
        ++off;
      }
    }
    __syncthreads();
    list_product<T, NT>(Q, n, lds_idx2, lds_val2, total, part,
                        [&](int64_t i, T sum) { g[i] = P.q[i * P.qs] + sum; });
    rows += total;
  };

  int status = NNLS_MAXITER_DEV;
  int it = 0;
  bool fresh = (P.y0 == nullptr);  // cold start: grad = q is exact
  if (P.y0) {
    refresh_gradient();
    fresh = true;
  }
  {
    int nf = nonfinite;
    T v = block_sum<T, NT>((T)nf, redT);
    if (v > (T)0) status = NNLS_NONFINITE_DEV;
  }
  double r_final = 0.0;

  while (status != NNLS_NONFINITE_DEV) {
    // Passive set, masked gradient and residual at the current iterate.
    int cnt = 0;
    T num = 0, res = 0;
    int bad = 0;
    for (int64_t i = tid; i < n; i += NT) {
      const T yi = y[i], gi = g[i];
      bad |= !is_finite_val(yi) || !is_finite_val(gi);
      const bool pas = (yi > (T)0) || (gi < (T)0);
      cnt += pas;
      const T pi = pas ? gi : (T)0;
      num += pi * pi;
      const T m = yi < gi ? yi : gi;
      res += m * m;
    }
    int total;
    int off = block_exclusive_scan<NT>(cnt, redI, total);
    for (int64_t i = tid; i < n; i += NT) {
      const T yi = y[i], gi = g[i];
      if ((yi > (T)0) || (gi < (T)0)) {
        lds_idx[off] = (int)i;
        lds_val[off] = gi;
        ++off;
      }
    }
    num = block_sum<T, NT>(num, redT);
    res = block_sum<T, NT>(res, redT);
    const T badv = block_sum<T, NT>((T)bad, redT);
    if (badv > (T)0) {
      status = NNLS_NONFINITE_DEV;
      break;
    }
    const double r = (double)(sqrt(res) / scale);
    r_final = r;
    if (P.trace != nullptr && tid == 0 && it < P.trace_len) {
      P.trace[2 * it] = (float)r;
      P.trace[2 * it + 1] = (float)num;
    }
    if (total == 0 || r <= tol) {
      if (fresh) {
        status = NNLS_CONVERGED_DEV;
        break;
      }
      refresh_gradient();
      fresh = true;
      continue;
    }
    if (it >= max_iter) {
      if (!fresh) {
        refresh_gradient();
        fresh = true;
        continue;
      }
      status = NNLS_MAXITER_DEV;
      break;
    }

    // Line-search product w = Q gbar over the passive rows; den = gbar^T w.
    rows += total;
    T den = 0;
    list_product<T, NT>(Q, n, lds_idx, lds_val, total, part, [&](int64_t i, T w) {
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      den += pi * w;
      P.w[i] = w;
    });
    den = block_sum<T, NT>(den, redT);
    if (!(den > (T)0) || !is_finite_val(den)) {
      status = NNLS_BREAKDOWN_DEV;
      break;
    }
    const T alpha = num / den;

    // Projected update and clipped set.
    int ccnt = 0;
    for (int64_t i = tid; i < n; i += NT) {
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      const T v = yi - alpha * pi;
      ccnt += (v < (T)0);
    }
    int ctotal;
    int coff = block_exclusive_scan<NT>(ccnt, redI, ctotal);
    for (int64_t i = tid; i < n; i += NT) {
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      const T v = yi - alpha * pi;
      if (v < (T)0) {
        lds_idx2[coff] = (int)i;
        lds_val2[coff] = alpha * pi - yi;  // delta = (0 - y) + alpha * gbar
        ++coff;
      }
    }
    __syncthreads();
    // y' = [y - alpha gbar]_+, grad' = grad - alpha w + Q[:, C] delta_C
    auto step_entry = [&](int64_t i, T corr) {
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      const T v = yi - alpha * pi;
      y[i] = v > (T)0 ? v : (T)0;
      g[i] = (gi - alpha * P.w[i]) + corr;
    };
    if (ctotal > 0) {
      list_product<T, NT>(Q, n, lds_idx2, lds_val2, ctotal, part, step_entry);
    } else {
      for (int64_t i = tid; i < n; i += NT) step_entry(i, (T)0);
      __syncthreads();
    }
    rows += ctotal;
    ++it;
    fresh = false;
  }

  for (int64_t i = tid; i < n; i += NT) {
    const T yi = y[i];
    P.x[i * P.qs] = P.s ? (T)((double)yi / P.s[i]) : yi;
  }
  if (tid == 0) {
    *iters_out = it;
    *kkt_out = status == NNLS_NONFINITE_DEV ? __builtin_nan("") : r_final;
    *status_out = status;
    if (rows_out) *rows_out = rows;
  }
}

// Byte offsets of the dynamic LDS of one workgroup of NT threads: the compacted passive list
// (values, indices), the clipped list (values, indices), the partial sums of list_product and
// the block-reduction scratch, each 16-byte aligned.
struct SwLdsLayout {
  size_t val, val2, idx, idx2, part, redT, redI, total;
};

__host__ __device__ inline size_t sw_align16(size_t v) { return (v + 15) & ~(size_t)15; }

__host__ __device__ inline SwLdsLayout sw_lds_layout(int64_t n, size_t elem, int nt) {
  SwLdsLayout L;
  L.val = 0;
  L.val2 = sw_align16(L.val + elem * n);
  L.idx = sw_align16(L.val2 + elem * n);
  L.idx2 = sw_align16(L.idx + sizeof(int) * n);
  L.part = sw_align16(L.idx2 + sizeof(int) * n);
  L.redT = sw_align16(L.part + elem * (size_t)(nt / kWave) * LP_CH);
  L.redI = sw_align16(L.redT + elem * (nt / kWave));
  L.total = sw_align16(L.redI + sizeof(int) * (nt / kWave));
  return L;
}

}  // namespace nnls
