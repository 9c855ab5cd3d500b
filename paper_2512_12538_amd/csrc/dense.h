// Work-group cooperative dense kernels shared by several translation units.
#pragma once

#include "common.h"

// In-place inverse of the n x n column-major complex matrix A (n <= 256) by
// Gauss-Jordan elimination with partial (row) pivoting; row interchanges are
// undone as column interchanges at the end.  Every thread of the block must
// call it.  A pivot step is three barriers: the first wave finds the pivot
// (largest modulus at or below the diagonal, first on ties) with shuffles;
// every thread then stages the new pivot row, the old row kk and the
// multipliers in shared memory from the values before the step; finally every
// element is updated from the staged values, the interchange folded in.
// Scratch (shared memory): rowk[n], rold[n], fcol[n], perm[n].  On a zero pivot
// *flag (shared) is set to (step + 1) and the elimination continues with a zero
// reciprocal, so the caller can report a singular matrix.
template <int NT>
__device__ void gj_inverse_inplace(double2* A, int n, double2* rowk, double2* rold, double2* fcol, int* perm,
                                   int* s_piv, int* flag) {
  const int tid = threadIdx.x;
  // element (i, c) of this thread's first slot and the stride between slots
  const int i0 = tid % n, c0 = tid / n, di = NT % n, dc = NT / n;
  for (int kk = 0; kk < n; ++kk) {
    if (tid < 64) {
      double best = -1.0;
      int bi = kk;
      for (int i = kk + tid; i < n; i += 64) {
        const double a = cabs2(A[i + (long long)kk * n]);
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
    const double2 pv = A[p + (long long)kk * n];
    const bool zero = cabs2(pv) == 0.0;
    if (tid == 0 && zero && *flag == 0) *flag = kk + 1;
    const double2 inv = zero ? mk(0.0, 0.0) : cdiv(mk(1.0, 0.0), pv);
    for (int c = tid; c < n; c += NT) {
      const double2 rk = A[kk + (long long)c * n], rp = A[p + (long long)c * n];
      rold[c] = rk;
      rowk[c] = (c == kk) ? inv : cmul(rp, inv);
    }
    for (int i = tid; i < n; i += NT) {
      const double2 v = (i == p) ? A[kk + (long long)kk * n] : A[i + (long long)kk * n];
      fcol[i] = (i == kk) ? mk(0.0, 0.0) : v;
    }
    __syncthreads();
    int i = i0, c = c0;
    while (c < n) {
      const long long e = i + (long long)c * n;
      if (i == kk) {
        A[e] = rowk[c];
      } else {
        const double2 base = (c == kk) ? mk(0.0, 0.0) : (i == p ? rold[c] : A[e]);
        A[e] = csub(base, cmul(fcol[i], rowk[c]));
      }
      i += di;
      c += dc;
      if (i >= n) {
        i -= n;
        c += 1;
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
