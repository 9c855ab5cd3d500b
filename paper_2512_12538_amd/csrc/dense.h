// Work-group cooperative dense kernels shared by several translation units.
#pragma once

#include "common.h"

// In-place inverse of the n x n column-major complex matrix A (n <= NT) by
// Gauss-Jordan elimination with partial (row) pivoting, by panels of NB
// pivots; row interchanges are undone as column interchanges at the end.
// Every thread of the block must call it.  A panel's NB columns are
// eliminated in shared memory (pivot: largest modulus at or below the
// diagonal, first on ties, found by the first wave with shuffles), the row
// interchanges applied to the whole matrix as they are chosen; the other
// columns then take the panel's NB eliminations at once.  Those eliminations
// compose to
//   x <- (x with rows K set to zero) + P x_K,
// K the panel's pivot rows, x_K the column's entries in those rows and P the
// panel's final columns, so the matrix is read and written once per panel
// instead of once per pivot.  Shared memory: pan[NB n], xk[NB n], fcol[n],
// rowk[NB] (double2), perm[n] (int).  On a zero pivot *flag (shared) is set
// to (step + 1) and the elimination continues with a zero reciprocal, so the
// caller can report a singular matrix.
template <int NT, int NB>
__device__ void gj_inverse_blocked(double2* A, int n, double2* pan, double2* xk, double2* fcol, double2* rowk,
                                   int* perm, int* s_piv, int* flag) {
  const int tid = threadIdx.x;
  // element (i, c) of this thread's first slot and the stride between slots
  const int i0 = tid % n, c0 = tid / n, di = NT % n, dc = NT / n;
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
        double best = -1.0;
        int bi = kk;
        for (int i = kk + tid; i < n; i += 64) {
          const double a = cabs2(col[i]);
          if (a > best) { best = a; bi = i; }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double ob = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (tid == 0) {
          *s_piv = bi;
          perm[kk] = bi;
        }
      }
      __syncthreads();
      const int p = *s_piv;
      if (p != kk) {
        for (int c = tid; c < n; c += NT) {
          double2* x = (c >= k0 && c < k0 + kb) ? pan + (c - k0) * n : A + (long long)c * n;
          const double2 v = x[kk];
          x[kk] = x[p];
          x[p] = v;
        }
        __syncthreads();
      }
      const double2 pv = col[kk];
      const bool zero = cabs2(pv) == 0.0;
      if (tid == 0 && zero && *flag == 0) *flag = kk + 1;
      const double2 inv = zero ? mk(0.0, 0.0) : cdiv(mk(1.0, 0.0), pv);
      for (int i = tid; i < n; i += NT) fcol[i] = (i == kk) ? mk(0.0, 0.0) : col[i];
      for (int c = tid; c < kb; c += NT) rowk[c] = (c == t) ? inv : cmul(pan[c * n + kk], inv);
      __syncthreads();
      int i = i0, c = c0;
      while (c < kb) {
        const int e = i + c * n;
        if (i == kk) {
          pan[e] = rowk[c];
        } else {
          const double2 base = (c == t) ? mk(0.0, 0.0) : pan[e];
          pan[e] = csub(base, cmul(fcol[i], rowk[c]));
        }
        i += di;
        c += dc;
        if (i >= n) { i -= n; c += 1; }
      }
      __syncthreads();
    }
    {
      // panel columns back to memory; the pivot rows of the other columns
      int i = i0, c = c0;
      while (c < kb) {
        A[i + (long long)(k0 + c) * n] = pan[i + c * n];
        i += di;
        c += dc;
        if (i >= n) { i -= n; c += 1; }
      }
      for (int e = tid; e < kb * n; e += NT) {
        const int t = e / n, cc = e - t * n;
        xk[e] = (cc >= k0 && cc < k0 + kb) ? mk(0.0, 0.0) : A[(k0 + t) + (long long)cc * n];
      }
    }
    __syncthreads();
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
        for (int t = 0; t < NB; ++t)
          if (t < kb) v = cfma(pr[t], xk[t * n + c], v);
        *a = v;
      }
    }
    __syncthreads();
  }
  for (int kk = n - 1; kk >= 0; --kk) {
    const int pr = perm[kk];
    if (pr != kk) {
      for (int i = tid; i < n; i += NT) {
        const double2 t = A[i + (long long)kk * n];
        A[i + (long long)kk * n] = A[i + (long long)pr * n];
        A[i + (long long)pr * n] = t;
      }
    }
    __syncthreads();
  }
}
