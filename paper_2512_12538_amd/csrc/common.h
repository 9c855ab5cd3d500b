// Shared device-side definitions: complex arithmetic on double2/float2, the
// per-box descriptor used by every batched kernel, and the cell-assembled
// 5-point impedance Helmholtz stencil of a box.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

typedef double2 c128;
typedef float2 c64;

template <typename T> struct cvec;
template <> struct cvec<double> { typedef double2 type; };
template <> struct cvec<float> { typedef float2 type; };

__host__ __device__ __forceinline__ double2 mk(double re, double im) { return make_double2(re, im); }
__host__ __device__ __forceinline__ float2 mk(float re, float im) { return make_float2(re, im); }
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a*b
__host__ __device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
__host__ __device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  return mk(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
// acc + conj(a)*b
__host__ __device__ __forceinline__ double2 cfmac(double2 a, double2 b, double2 acc) {
  return mk(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}
__host__ __device__ __forceinline__ double2 cconj(double2 a) { return mk(a.x, -a.y); }
__host__ __device__ __forceinline__ float2 cconj(float2 a) { return mk(a.x, -a.y); }
__host__ __device__ __forceinline__ double2 cscale(double2 a, double s) { return mk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return mk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ __forceinline__ float2 to_c64(double2 a) { return mk((float)a.x, (float)a.y); }
__device__ __forceinline__ double2 to_c128(float2 a) { return mk((double)a.x, (double)a.y); }
__device__ __forceinline__ double2 to_c128(double2 a) { return a; }
template <typename T> __device__ __forceinline__ typename cvec<T>::type from_c128(double2 a);
template <> __device__ __forceinline__ double2 from_c128<double>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_c128<float>(double2 a) { return to_c64(a); }

// Work-group barrier that orders LDS accesses only: outstanding global loads
// (prefetches) stay in flight across it, unlike __syncthreads().  Valid only
// where threads exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Box descriptor shared by all batched kernels of one level.  All node ranges
// are inclusive global node coordinates (p along x, q along y); a box's local
// vector is p-major: local index (p - p0) * ny + (q - q0).
struct BoxDev {
  int p0, p1, q0, q1;     // nodes of the box
  int op0, op1, oq0, oq1; // nodes kept by the restricted prolongation P_i
  int nx, ny, n;          // nodes per side, total
  int parent;             // index of the parent box in the level above
  int pp0, pq0, pny;      // parent's origin and width (for local indexing)
  int m_in;               // interface nodes
  int if_off;             // offset into the level's interface-index table
  int r, s;               // coarse rank and sketch width of this box
  int cidx;               // first column of this box's block in its parent's coarse matrix
  int n_own;              // owned nodes (op1-op0+1)*(oq1-oq0+1)
  int own_ny;             // owned width in q
  int tr_off, tr_cnt;     // trace rows of the interface map of this box
  int adj_off, adj_cnt;   // adjoint-trace entries (CSR over owned nodes)
  int prob;               // problem of the box (row of the operator table)
  long long voff;         // node offset of this box in a level buffer
  long long goff;         // offset (in complex entries) of this box's block factors
  long long coff;         // offset (in complex entries) of this box's coarse block C_i
  long long acoff;        // offset of the Galerkin product A C_i (dilated owned box)
};

// Parent-problem descriptor (a box that has children), one per box of a level
// that carries a coarse space.
struct ParentDev {
  int n_c;            // coarse dimension sum_i r_i
  int child0, nchild; // children range in the level below
  int pad;
  long long aoff;     // offset of its A_c^{-1} (n_c x n_c, column-major)
  long long yoff;     // offset of its coarse vectors (n_c entries per rhs)
};

// Operator description in device memory.
struct OpDev {
  const double* k; // wavenumber per global node, or null for the constant
  double kc;
  double h, ih2;   // h = 1/N, 1/h^2
  int N1;          // nodes per side (N+1)
  int dim;
};

__device__ __forceinline__ double op_k(const OpDev& o, int p, int q) {
  return o.k ? o.k[(long long)p * (o.dim == 2 ? o.N1 : 1) + q] : o.kc;
}

// Entry of the cell-assembled box matrix A_D in row (p, q) and column
// (p + dp, q + dq), dp, dq in {-1, 0, 1} with |dp| + |dq| <= 1, for the box
// [p0, p1] x [q0, q1].  The caller guarantees both nodes are inside the box.
// Edges carry (cells next to the edge)/(2 h^2); each node gets -k^2/4 per
// cell and -i k/(2h) per boundary edge of the box (1D: cells and edges are
// counted as if the box had two cells across, which gives the 3-point rows).
__device__ __forceinline__ double2 stencil_coef(const OpDev& o, int p0, int p1, int q0, int q1,
                                                 int p, int q, int dp, int dq) {
  const double cx = (double)((p > p0) + (p < p1));
  const double cy = o.dim == 2 ? (double)((q > q0) + (q < q1)) : 2.0;
  if (dp != 0) return mk(-0.5 * cy * o.ih2, 0.0);
  if (dq != 0) return mk(-0.5 * cx * o.ih2, 0.0);
  const double kk = op_k(o, p, q);
  double stiff = 0.5 * cx * cy * o.ih2;
  if (o.dim == 2) stiff *= 2.0;
  double nb = (p == p0 || p == p1) ? cy : 0.0;
  if (o.dim == 2 && (q == q0 || q == q1)) nb += cx;
  return mk(stiff - 0.25 * kk * kk * cx * cy, -0.5 * kk * nb / o.h);
}
