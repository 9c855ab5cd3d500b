// Work-group cooperative dense kernels shared by several translation units.
#pragma once

#include "common.h"

// In-place inverse of the n x n column-major complex matrix A by Gauss-Jordan
// elimination with partial (row) pivoting; row interchanges are undone as
// column interchanges at the end.  Every thread of the block must call it.
// Scratch (shared memory): fcol[n], perm[n], rv[NT], ri[NT].  On a zero pivot
// *flag (shared) is set to (step + 1) and the elimination continues with a
// zero reciprocal, so the caller can report a singular matrix.
template <int NT>
__device__ void gj_inverse_inplace(double2* A, int n, double2* fcol, int* perm, double* rv, int* ri,
                                   double2* s_inv, int* flag) {
  const int tid = threadIdx.x;
  for (int kk = 0; kk < n; ++kk) {
    double best = -1.0;
    int bi = kk;
    for (int i = kk + tid; i < n; i += NT) {
      const double a = cabs2(A[i + (long long)kk * n]);
      if (a > best) { best = a; bi = i; }
    }
    rv[tid] = best;
    ri[tid] = bi;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
      if (tid < st) {
        const double o = rv[tid + st];
        const int oi = ri[tid + st];
        if (o > rv[tid] || (o == rv[tid] && oi < ri[tid])) { rv[tid] = o; ri[tid] = oi; }
      }
      __syncthreads();
    }
    const int pr = ri[0];
    if (tid == 0) perm[kk] = pr;
    if (pr != kk) {
      for (int c = tid; c < n; c += NT) {
        const double2 t = A[kk + (long long)c * n];
        A[kk + (long long)c * n] = A[pr + (long long)c * n];
        A[pr + (long long)c * n] = t;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const double2 pv = A[kk + (long long)kk * n];
      if (cabs2(pv) == 0.0) {
        if (*flag == 0) *flag = kk + 1;
        *s_inv = mk(0.0, 0.0);
      } else {
        *s_inv = cdiv(mk(1.0, 0.0), pv);
      }
    }
    __syncthreads();
    const double2 inv = *s_inv;
    for (int c = tid; c < n; c += NT) {
      const long long e = kk + (long long)c * n;
      A[e] = (c == kk) ? inv : cmul(A[e], inv);
    }
    for (int i = tid; i < n; i += NT) fcol[i] = (i == kk) ? mk(0.0, 0.0) : A[i + (long long)kk * n];
    __syncthreads();
    for (long long e = tid; e < (long long)n * n; e += NT) {
      const int i = (int)(e % n), c = (int)(e / n);
      if (i == kk) continue;
      const double2 rowk = A[kk + (long long)c * n];
      const double2 base = (c == kk) ? mk(0.0, 0.0) : A[e];
      A[e] = csub(base, cmul(fcol[i], rowk));
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
