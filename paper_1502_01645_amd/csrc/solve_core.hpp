// Device code of Algorithm 2 for one right-hand side handled by one workgroup: shared by the
// per-column solver and the uneven-batch solver.
//
// The workgroup owns one column: y, the gradient and Q*gbar live in caller-provided global
// vectors, the masked gradient and the compacted passive / clipped index lists live in LDS.
// Because Q is symmetric, the product Q * gbar only needs the rows of Q in the passive set
// (each a contiguous row), and the incremental gradient reuses it:
//     grad' = grad + Q (y' - y) = grad - alpha * (Q gbar) + Q[:, C] delta_C,
// where C is the set of entries the projection clipped and delta = (y' - y) + alpha * gbar is
// nonzero only there.  Threads own output entries i; each passive row j is read once, coalesced.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace nnls {

constexpr int SW_NT = 256;

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

// sum over the compacted list (idx, val) of val_m * Q[idx_m, i]: row idx_m of Q is read at
// column i, so consecutive threads read consecutive addresses of one row.
template <typename T>
__device__ __forceinline__ T row_combo(const T* __restrict__ Q, int64_t n, int64_t i,
                                       const int* __restrict__ idx, const T* __restrict__ val,
                                       int cnt) {
  T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int m = 0;
  for (; m + 3 < cnt; m += 4) {
    const int j0 = idx[m], j1 = idx[m + 1], j2 = idx[m + 2], j3 = idx[m + 3];
    a0 += val[m] * Q[(int64_t)j0 * n + i];
    a1 += val[m + 1] * Q[(int64_t)j1 * n + i];
    a2 += val[m + 2] * Q[(int64_t)j2 * n + i];
    a3 += val[m + 3] * Q[(int64_t)j3 * n + i];
  }
  for (; m < cnt; ++m) a0 += val[m] * Q[(int64_t)idx[m] * n + i];
  return (a0 + a1) + (a2 + a3);
}

template <typename T>
__device__ void solve_column(const SolveCol<T>& P, double tol, int max_iter, int32_t* iters_out,
                             double* kkt_out, int32_t* status_out, int64_t* rows_out,
                             T* lds_val, int* lds_idx,
                             T* lds_val2, int* lds_idx2, T* redT, int* redI) {
  const int tid = threadIdx.x;
  const int64_t n = P.n;
  const T* __restrict__ Q = P.Q;
  T* __restrict__ y = P.y;
  T* __restrict__ g = P.g;

  // ||q|| for the relative residual; start point.
  T qq = 0;
  int nonfinite = 0;
  for (int64_t i = tid; i < n; i += SW_NT) {
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
  qq = block_sum<T, SW_NT>(qq, redT);
  const T qnorm = sqrt(qq);
  const T scale = qnorm > (T)0 ? qnorm : (T)1;
  __syncthreads();

  int64_t rows = 0;  // rows of Q read by the products
  // Recompute grad = Q y + q exactly over the rows with y_j > 0.
  auto refresh_gradient = [&]() {
    int cnt = 0;
    for (int64_t i = tid; i < n; i += SW_NT) cnt += (y[i] > (T)0);
    int total;
    int off = block_exclusive_scan<SW_NT>(cnt, redI, total);
    for (int64_t i = tid; i < n; i += SW_NT) {
      const T yi = y[i];
      if (yi > (T)0) {
        lds_idx2[off] = (int)i;
        lds_val2[off] = yi;
        ++off;
      }
    }
    __syncthreads();
    for (int64_t i = tid; i < n; i += SW_NT)
      g[i] = P.q[i * P.qs] + row_combo(Q, n, i, lds_idx2, lds_val2, total);
    rows += total;
    __syncthreads();
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
    T v = block_sum<T, SW_NT>((T)nf, redT);
    if (v > (T)0) status = NNLS_NONFINITE_DEV;
  }
  double r_final = 0.0;

  while (status != NNLS_NONFINITE_DEV) {
    // Passive set, masked gradient and residual at the current iterate.
    int cnt = 0;
    T num = 0, res = 0;
    int bad = 0;
    for (int64_t i = tid; i < n; i += SW_NT) {
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
    int off = block_exclusive_scan<SW_NT>(cnt, redI, total);
    for (int64_t i = tid; i < n; i += SW_NT) {
      const T yi = y[i], gi = g[i];
      if ((yi > (T)0) || (gi < (T)0)) {
        lds_idx[off] = (int)i;
        lds_val[off] = gi;
        ++off;
      }
    }
    num = block_sum<T, SW_NT>(num, redT);
    res = block_sum<T, SW_NT>(res, redT);
    const T badv = block_sum<T, SW_NT>((T)bad, redT);
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
    for (int64_t i = tid; i < n; i += SW_NT) {
      const T w = row_combo(Q, n, i, lds_idx, lds_val, total);
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      den += pi * w;
      P.w[i] = w;
    }
    den = block_sum<T, SW_NT>(den, redT);
    if (!(den > (T)0) || !is_finite_val(den)) {
      status = NNLS_BREAKDOWN_DEV;
      break;
    }
    const T alpha = num / den;

    // Projected update and clipped set.
    int ccnt = 0;
    for (int64_t i = tid; i < n; i += SW_NT) {
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      const T v = yi - alpha * pi;
      ccnt += (v < (T)0);
    }
    int ctotal;
    int coff = block_exclusive_scan<SW_NT>(ccnt, redI, ctotal);
    for (int64_t i = tid; i < n; i += SW_NT) {
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
    for (int64_t i = tid; i < n; i += SW_NT) {
      const T yi = y[i], gi = g[i];
      const T pi = ((yi > (T)0) || (gi < (T)0)) ? gi : (T)0;
      const T v = yi - alpha * pi;
      const T w = P.w[i];
      T gn = gi - alpha * w;
      if (ctotal > 0) gn += row_combo(Q, n, i, lds_idx2, lds_val2, ctotal);
      y[i] = v > (T)0 ? v : (T)0;
      g[i] = gn;
    }
    rows += ctotal;
    __syncthreads();
    ++it;
    fresh = false;
  }

  for (int64_t i = tid; i < n; i += SW_NT) {
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

// Byte offsets of the dynamic LDS of one workgroup: the compacted passive list (values, indices),
// the clipped list (values, indices) and the block-reduction scratch, each 16-byte aligned.
struct SwLdsLayout {
  size_t val, val2, idx, idx2, redT, redI, total;
};

__host__ __device__ inline size_t sw_align16(size_t v) { return (v + 15) & ~(size_t)15; }

__host__ __device__ inline SwLdsLayout sw_lds_layout(int64_t n, size_t elem) {
  SwLdsLayout L;
  L.val = 0;
  L.val2 = sw_align16(L.val + elem * n);
  L.idx = sw_align16(L.val2 + elem * n);
  L.idx2 = sw_align16(L.idx + sizeof(int) * n);
  L.redT = sw_align16(L.idx2 + sizeof(int) * n);
  L.redI = sw_align16(L.redT + elem * (SW_NT / kWave));
  L.total = sw_align16(L.redI + sizeof(int) * (SW_NT / kWave));
  return L;
}

}  // namespace nnls
