// Gauss-Jordan inversion of a small dense complex matrix held in the
// registers of one NT-thread work-group, with partial row pivoting.  Thread
// t owns row i = t % n and the columns c = g + G r (g = t / n, G = NT / n,
// r < RE), so row quantities are per-thread scalars and no index division
// happens in the elimination loop.  LDS carries only the pivot column, the two
// rows being interchanged, the pivot's reciprocal (computed once, by one
// thread) and the interchange record: a pivot step costs three barriers and
// no global memory traffic.
#pragma once

#include "common.h"

namespace gjr {

struct Scratch {
  double2 colk[2][256];
  double2 rowk[2][256];
  double2 rowp[2][256];
  double2 inv[2];
  int perm[256];
  int pos[256];
  int piv[2];
  int flag;
  int bad;
};

struct Layout {
  int i, g, G;
  bool act;
};

template <int NT>
__device__ __forceinline__ Layout layout(int n) {
  Layout L;
  L.G = NT / n;
  L.i = threadIdx.x % n;
  L.g = threadIdx.x / n;
  L.act = L.g < L.G;
  return L;
}

// Inverts the n x n matrix held in A (n <= 256, n <= NT, ceil(n / (NT / n)) <=
// RE) in place up to the final column permutation: on return
// inverse[:, sc.pos[c]] = (held column c).  sc.flag must be zero on entry;
// it is set to (step + 1) at the first zero pivot.
template <int NT, int RE>
__device__ __forceinline__ void invert(double2 (&A)[RE], int n, const Layout& L, Scratch& sc) {
  const int tid = threadIdx.x;
  for (int kk = 0; kk < n; ++kk) {
    const int bsel = kk & 1;
    // A: publish column kk and row kk
    if (L.act) {
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int c = L.g + L.G * r;
        if (c < n) {
          if (c == kk) sc.colk[bsel][L.i] = A[r];
          if (L.i == kk) sc.rowk[bsel][c] = A[r];
        }
      }
    }
    lds_barrier();
    // B: pivot search (first wave): largest modulus at or below the diagonal, first on ties
    if (tid < 64) {
      double best = -1.0;
      int bi = kk;
      for (int i = kk + tid; i < n; i += 64) {
        const double a = cabs2(sc.colk[bsel][i]);
        if (a > best) { best = a; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        sc.piv[bsel] = bi;
        sc.perm[kk] = bi;
        if (best <= 0.0 && sc.flag == 0) sc.flag = kk + 1;
        sc.inv[bsel] = best > 0.0 ? cdiv(mk(1.0, 0.0), sc.colk[bsel][bi]) : mk(0.0, 0.0);
      }
    }
    lds_barrier();
    const int p = sc.piv[bsel];
    // C: publish row p
    if (L.act && L.i == p) {
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int c = L.g + L.G * r;
        if (c < n) sc.rowp[bsel][c] = A[r];
      }
    }
    lds_barrier();
    // D: interchange rows kk and p, scale the pivot row, eliminate column kk elsewhere
    if (L.act) {
      const double2 inv = sc.inv[bsel];
      const bool is_k = L.i == kk, is_p = L.i == p;
      const double2 f = is_p ? sc.colk[bsel][kk] : sc.colk[bsel][L.i];
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int c = L.g + L.G * r;
        if (c < n) {
          const double2 newk = (c == kk) ? inv : cmul(sc.rowp[bsel][c], inv);
          if (is_k) {
            A[r] = newk;
          } else {
            const double2 old = is_p ? sc.rowk[bsel][c] : A[r];
            A[r] = csub((c == kk) ? mk(0.0, 0.0) : old, cmul(f, newk));
          }
        }
      }
    }
    // no barrier: the next step publishes into the other LDS buffer set
  }
  lds_barrier();
  // column interchanges undone in reverse order, as one permutation
  if (tid == 0) {
    int* idx = sc.pos;  // idx[t] = held column that ends at position t
    for (int c = 0; c < n; ++c) idx[c] = c;
    for (int kk = n - 1; kk >= 0; --kk) {
      const int pk = sc.perm[kk];
      const int t = idx[kk];
      idx[kk] = idx[pk];
      idx[pk] = t;
    }
    for (int t = 0; t < n; ++t) sc.perm[idx[t]] = t;
    for (int c = 0; c < n; ++c) sc.pos[c] = sc.perm[c];
  }
  lds_barrier();
}

// The same elimination with the diagonal pivots, one barrier per step.  The
// pivot ratio is watched without a reduction: the thread holding a(i, kk),
// i > kk, flags the step if ratio * |a_ik| > |a_kk|; a flagged inversion is
// discarded (returns false) and the caller repeats it with row interchanges.
// On success sc.pos is the identity.
template <int NT, int RE>
__device__ __forceinline__ bool invert_diag(double2 (&A)[RE], int n, const Layout& L, Scratch& sc, double ratio) {
  const int tid = threadIdx.x;
  if (tid == 0) sc.bad = 0;
  const double r2 = ratio * ratio;
  for (int kk = 0; kk < n; ++kk) {
    const int bsel = kk & 1;
    if (L.act) {
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int c = L.g + L.G * r;
        if (c < n) {
          if (c == kk) sc.colk[bsel][L.i] = A[r];
          if (L.i == kk) sc.rowk[bsel][c] = A[r];
          if (c == kk && L.i == kk) sc.inv[bsel] = cabs2(A[r]) > 0.0 ? cdiv(mk(1.0, 0.0), A[r]) : mk(0.0, 0.0);
        }
      }
    }
    lds_barrier();
    const double2 pv = sc.colk[bsel][kk];
    const double pa = cabs2(pv);
    if (tid == 0 && !(pa > 0.0)) sc.bad = 1;
    if (L.act) {
      const double2 inv = sc.inv[bsel];
      const bool is_k = L.i == kk;
      const double2 f = sc.colk[bsel][L.i];
      if (L.i > kk && L.g == kk % L.G && !(r2 * cabs2(f) <= pa)) sc.bad = 1;
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int c = L.g + L.G * r;
        if (c < n) {
          const double2 newk = (c == kk) ? inv : cmul(sc.rowk[bsel][c], inv);
          if (is_k) A[r] = newk;
          else A[r] = csub((c == kk) ? mk(0.0, 0.0) : A[r], cmul(f, newk));
        }
      }
    }
  }
  if (tid < n) sc.pos[tid] = tid;
  lds_barrier();
  return sc.bad == 0;
}

}  // namespace gjr
