// Work-group cooperative dense kernels shared by several translation units.
#pragma once

#include "common.h"

// In-place inverse of the n x n column-major complex matrix A (n <= NT) by
// Gauss-Jordan elimination with partial (row) pivoting, by panels of NB
// pivots.  Every thread of the block must call it.
//
// A panel's NB columns are eliminated in shared memory, two barriers a pivot:
// the first wave finds the pivot (largest modulus at or below the diagonal,
// first on ties) with shuffles and stages the step (reciprocal, scaled pivot
// row, multipliers), then every thread updates the panel, the interchange of
// rows kk and p folded in.  For the other columns the panel's interchanges
// are only recorded (src[r]: the row whose entry now belongs in row r).  At
// the end of the panel every other column x takes them, then the panel's NB
// eliminations at once, which compose to
//   x <- (x with rows K set to zero) + P x_K,
// K the panel's pivot rows, x_K the column's (interchanged) entries in those
// rows and P the panel's final columns; the matrix is read and written once
// per panel and no global memory access waits inside the pivot loop.  A row
// outside K ends with the entry of a row of K (its own entry moved into K the
// first time it was chosen), so the interchanges of such rows read only rows
// the update overwrites afterwards.  With tot the composite of all
// interchanges, the result X = (A with rows tot)^-1 gives A^-1 by the column
// scatter A^-1[:, tot[r]] = X[:, r], done by row blocks staged in shared
// memory.
//
// Shared memory: work[2 NB n], fcol[n], rowk[NB], rold[NB] (double2);
// src[n], tot[n], perm[NB] (int).  On a zero pivot *flag (shared) is set to
// (step + 1) and the elimination continues with a zero reciprocal, so the
// caller can report a singular matrix.
template <int NT, int NB>
__device__ void gj_inverse_blocked(double2* A, int n, double2* work, double2* fcol, double2* rowk, double2* rold,
                                   int* src, int* tot, int* perm, int* s_piv, int* s_any, int* flag) {
  const int tid = threadIdx.x;
  double2* pan = work;           // NB x n, column-major: the panel's columns
  double2* xk = work + NB * n;   // NB x n: xk[t n + c] = entry (k0 + t, c)
  // element (i, c) of this thread's first slot and the stride between slots
  const int i0 = tid % n, c0 = tid / n, di = NT % n, dc = NT / n;
  for (int i = tid; i < n; i += NT) {
    src[i] = i;
    tot[i] = i;
  }
  if (tid == 0) *s_any = 0;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = n - k0 < NB ? n - k0 : NB;
    {
      int i = i0, c = c0;
      while (c < kb) {
        pan[i + c * n] = A[i + (long long)(k0 + c) * n];
        i += di;
        c += dc;
        if (i >= n) { i -= n; c += 1; }
      }
    }
    __syncthreads();
    for (int t = 0; t < kb; ++t) {
      const int kk = k0 + t;
      const double2* col = pan + t * n;
      if (tid < 64) {
        // the first wave finds the pivot and stages the step: pivot row
        // (scaled), old row kk and the multipliers of the interchanged column
        double best = -1.0;
        int p = kk;
        for (int i = kk + tid; i < n; i += 64) {
          const double a = cabs2(col[i]);
          if (a > best) { best = a; p = i; }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double ob = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(p, o, 64);
          if (ob > best || (ob == best && oi < p)) { best = ob; p = oi; }
        }
        const double2 pv = col[p];
        const bool zero = cabs2(pv) == 0.0;
        const double2 inv = zero ? mk(0.0, 0.0) : cdiv(mk(1.0, 0.0), pv);
        for (int c = tid; c < kb; c += 64) {
          rold[c] = pan[c * n + kk];
          rowk[c] = (c == t) ? inv : cmul(pan[c * n + p], inv);
        }
        for (int i = tid; i < n; i += 64) fcol[i] = (i == kk) ? mk(0.0, 0.0) : (i == p ? col[kk] : col[i]);
        if (tid == 0) {
          *s_piv = p;
          perm[t] = p;
          if (zero && *flag == 0) *flag = kk + 1;
          if (p != kk) {
            *s_any = 1;
            int v = src[kk];
            src[kk] = src[p];
            src[p] = v;
            v = tot[kk];
            tot[kk] = tot[p];
            tot[p] = v;
          }
        }
      }
      __syncthreads();
      const int p = *s_piv;
      int i = i0, c = c0;
      while (c < kb) {
        const int e = i + c * n;
        if (i == kk) {
          pan[e] = rowk[c];
        } else {
          const double2 base = (c == t) ? mk(0.0, 0.0) : (i == p ? rold[c] : pan[e]);
          pan[e] = csub(base, cmul(fcol[i], rowk[c]));
        }
        i += di;
        c += dc;
        if (i >= n) { i -= n; c += 1; }
      }
      __syncthreads();
    }
    {
      // panel columns back to memory; the other columns take the panel's
      // interchanges: rows K staged in xk, rows outside K written in place
      int i = i0, c = c0;
      while (c < kb) {
        A[i + (long long)(k0 + c) * n] = pan[i + c * n];
        i += di;
        c += dc;
        if (i >= n) { i -= n; c += 1; }
      }
      for (int cc = tid; cc < n; cc += NT) {
        if (cc >= k0 && cc < k0 + kb) continue;
        double2* x = A + (long long)cc * n;
        for (int t = 0; t < kb; ++t) xk[t * n + cc] = x[src[k0 + t]];
        for (int t = kb; t < NB; ++t) xk[t * n + cc] = mk(0.0, 0.0);
        __threadfence_block();
        for (int t = 0; t < kb; ++t) {
          const int r = perm[t];
          if (r >= k0 + kb) x[r] = x[src[r]];
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < n; r += NT) src[r] = r;
    // trailing update: thread = one row i0 (its panel row in registers),
    // columns c0, c0 + NT / n, ...
    if (c0 < dc) {
      double2 pr[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) pr[t] = t < kb ? pan[t * n + i0] : mk(0.0, 0.0);
      const bool inK = i0 >= k0 && i0 < k0 + kb;
      for (int c = c0; c < n; c += dc) {
        if (c >= k0 && c < k0 + kb) continue;
        double2* a = A + i0 + (long long)c * n;
        double2 v = inK ? mk(0.0, 0.0) : *a;
#pragma unroll
        for (int t = 0; t < NB; ++t) v = cfma(pr[t], xk[t * n + c], v);
        *a = v;
      }
    }
    __syncthreads();
  }
  if (*s_any == 0) return;
  // A^-1[:, tot[r]] = X[:, r], by blocks of 2 NB rows staged in work
  constexpr int R = 2 * NB;
  for (int r0 = 0; r0 < n; r0 += R) {
    for (int e = tid; e < R * n; e += NT) {
      const int r = e % R, j = e / R;
      if (r0 + r < n) work[e] = A[(r0 + r) + (long long)j * n];
    }
    __syncthreads();
    for (int e = tid; e < R * n; e += NT) {
      const int r = e % R, j = e / R;
      if (r0 + r < n) A[(r0 + r) + (long long)tot[j] * n] = work[e];
    }
    __syncthreads();
  }
}
