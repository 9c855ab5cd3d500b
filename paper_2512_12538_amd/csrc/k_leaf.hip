// Leaf subdomain solves A~_i x = b (the local impedance problems of eq. (sub1)).
//
// The box matrix in line-major order (line j = all nodes with p = p0 + j, the
// ny nodes of a line contiguous) is block tridiagonal: the diagonal blocks
// are tridiagonal, the couplings between neighbouring lines are diagonal.  The
// factorisation keeps the inverse Schur complements of the block LU
//   S_0 = A_00,  S_j = A_jj - A_{j,j-1} S_{j-1}^{-1} A_{j-1,j},  G_j = S_j^{-1},
// and a solve is one forward and one backward sweep over the lines, each step
// a dense (ny x ny) by (ny x q) product with the streamed G_j:
//   forward   w_j = G_j (b_j - A_{j,j-1} w_{j-1}),
//   backward  x_j = w_j - G_j A_{j,j+1} x_{j+1}.
// G_j is stored column-major, so consecutive threads (consecutive rows i)
// read consecutive addresses for a fixed column k.
#include "dense.h"
#include "kernels.h"

namespace {

constexpr int TB = 256;

__device__ __forceinline__ double2 diag_block(const OpDev& op, const BoxDev& B, int j, int i, int k) {
  const int p = B.p0 + j, q = B.q0 + i;
  if (i == k) return stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, q, 0, 0);
  if (op.dim == 2 && (k == i + 1 || k == i - 1)) return stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, q, 0, k - i);
  return mk(0.0, 0.0);
}

// In-place block LU of one leaf per work-group; each S_j inverted by
// Gauss-Jordan elimination with partial (row) pivoting.
__global__ void __launch_bounds__(TB) k_leaf_factor(OpDev op, const BoxDev* __restrict__ leaves,
                                                    c128* __restrict__ G, int* __restrict__ info) {
  const BoxDev B = leaves[blockIdx.x];
  const int b = B.ny;
  const int tid = threadIdx.x;
  extern __shared__ unsigned char smem_raw[];
  double2* fcol = reinterpret_cast<double2*>(smem_raw);           // b
  double* rv = reinterpret_cast<double*>(fcol + b);                // TB
  int* ri = reinterpret_cast<int*>(rv + TB);                        // TB
  int* perm = ri + TB;                                              // b
  __shared__ double2 s_inv;
  __shared__ int s_flag;
  if (tid == 0) s_flag = 0;
  for (int j = 0; j < B.nx; ++j) {
    c128* Gj = G + B.goff + (long long)j * b * b;
    const c128* Gp = G + B.goff + (long long)(j - 1) * b * b;
    // S_j = A_jj - A_{j,j-1} G_{j-1} A_{j-1,j}
    for (int e = tid; e < b * b; e += TB) {
      const int i = e % b, k = e / b;
      double2 v = diag_block(op, B, j, i, k);
      if (j > 0) {
        const double2 ai = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j, B.q0 + i, -1, 0);
        const double2 ak = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j - 1, B.q0 + k, 1, 0);
        v = csub(v, cmul(cmul(ai, Gp[e]), ak));
      }
      Gj[e] = v;
    }
    __syncthreads();
    int flag_before = s_flag;
    gj_inverse_inplace<TB>(Gj, b, fcol, perm, rv, ri, &s_inv, &s_flag);
    if (tid == 0 && flag_before == 0 && s_flag != 0) s_flag = j * b + s_flag;
    __syncthreads();
  }
  if (tid == 0 && info) info[blockIdx.x] = s_flag;
}

// Forward and backward sweeps for QB right-hand sides per work-group.
// Thread t works on row i = t % b of slice kap = t / b (K = TB / b slices
// split the inner dimension k); partial sums meet in LDS.
template <typename T, int QB>
__global__ void __launch_bounds__(TB) k_leaf_solve(OpDev op, const BoxDev* __restrict__ leaves, int q,
                                                   const typename cvec<T>::type* __restrict__ G,
                                                   const c128* __restrict__ rhs, c128* __restrict__ x) {
  typedef typename cvec<T>::type CT;
  const BoxDev B = leaves[blockIdx.x];
  const int b = B.ny;
  const int K = TB / b;
  const int tid = threadIdx.x;
  const int kap = tid / b, i = tid - kap * b;
  const bool act = kap < K;
  const int c0 = blockIdx.y * QB;
  extern __shared__ unsigned char smem_raw[];
  CT* y = reinterpret_cast<CT*>(smem_raw);  // b * QB
  CT* w = y + b * QB;                        // b * QB
  CT* red = w + b * QB;                      // K * b * QB
  const long long base = B.voff * q;
  // forward sweep
  for (int j = 0; j < B.nx; ++j) {
    for (int e = tid; e < b * QB; e += TB) {
      const int k = e % b, c = e / b;
      CT v = mk((T)0, (T)0);
      if (c0 + c < q) {
        double2 r = rhs[base + (long long)(c0 + c) * B.n + (long long)j * b + k];
        if (j > 0) {
          const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j, B.q0 + k, -1, 0);
          r = csub(r, cmul(a, to_c128(w[e])));
        }
        v = from_c128<T>(r);
      }
      y[e] = v;
    }
    __syncthreads();
    if (act) {
      CT acc[QB];
#pragma unroll
      for (int c = 0; c < QB; ++c) acc[c] = mk((T)0, (T)0);
      const CT* Gj = G + B.goff + (long long)j * b * b;
      for (int k = kap; k < b; k += K) {
        const CT g = Gj[(long long)k * b + i];
#pragma unroll
        for (int c = 0; c < QB; ++c) acc[c] = cfma(g, y[c * b + k], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < QB; ++c) red[(kap * QB + c) * b + i] = acc[c];
    }
    __syncthreads();
    for (int e = tid; e < b * QB; e += TB) {
      const int ii = e % b, c = e / b;
      CT s = red[c * b + ii];
      for (int kp = 1; kp < K; ++kp) s = cadd(s, red[(kp * QB + c) * b + ii]);
      w[e] = s;
      if (c0 + c < q) x[base + (long long)(c0 + c) * B.n + (long long)j * b + ii] = to_c128(s);
    }
    __syncthreads();
  }
  // backward sweep; w holds x_{j+1}
  for (int j = B.nx - 2; j >= 0; --j) {
    for (int e = tid; e < b * QB; e += TB) {
      const int k = e % b;
      const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j, B.q0 + k, 1, 0);
      y[e] = from_c128<T>(cmul(a, to_c128(w[e])));
    }
    __syncthreads();
    if (act) {
      CT acc[QB];
#pragma unroll
      for (int c = 0; c < QB; ++c) acc[c] = mk((T)0, (T)0);
      const CT* Gj = G + B.goff + (long long)j * b * b;
      for (int k = kap; k < b; k += K) {
        const CT g = Gj[(long long)k * b + i];
#pragma unroll
        for (int c = 0; c < QB; ++c) acc[c] = cfma(g, y[c * b + k], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < QB; ++c) red[(kap * QB + c) * b + i] = acc[c];
    }
    __syncthreads();
    for (int e = tid; e < b * QB; e += TB) {
      const int ii = e % b, c = e / b;
      CT s = red[c * b + ii];
      for (int kp = 1; kp < K; ++kp) s = cadd(s, red[(kp * QB + c) * b + ii]);
      double2 xv = mk(0.0, 0.0);
      if (c0 + c < q) {
        const long long at = base + (long long)(c0 + c) * B.n + (long long)j * b + ii;
        xv = csub(x[at], to_c128(s));
        x[at] = xv;
      }
      w[e] = from_c128<T>(xv);
    }
    __syncthreads();
  }
}

template <typename T, int QB>
hipError_t launch_solve_qb(const OpDev& op, const BoxDev* leaves, int nleaf, int max_ny, int q,
                           const typename cvec<T>::type* G, const c128* rhs, c128* x, hipStream_t s) {
  typedef typename cvec<T>::type CT;
  // y and w hold b*QB entries each; the partial sums K*b*QB <= TB*QB entries
  const size_t shm = sizeof(CT) * (size_t)QB * (2 * (size_t)max_ny + TB);
  dim3 grid(nleaf, (q + QB - 1) / QB);
  hipLaunchKernelGGL((k_leaf_solve<T, QB>), grid, dim3(TB), shm, s, op, leaves, q, G, rhs, x);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_factor(const OpDev& op, const BoxDev* leaves, int nleaf, int max_ny, c128* G,
                              int* info, hipStream_t s) {
  if (nleaf <= 0) return hipSuccess;
  const size_t shm = sizeof(double2) * max_ny + (sizeof(double) + sizeof(int)) * TB + sizeof(int) * max_ny;
  hipLaunchKernelGGL(k_leaf_factor, dim3(nleaf), dim3(TB), shm, s, op, leaves, G, info);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_leaf_solve(const OpDev& op, const BoxDev* leaves, int nleaf, int max_ny, int q,
                             const typename cvec<T>::type* G, const c128* rhs, c128* x, hipStream_t s) {
  if (nleaf <= 0 || q <= 0) return hipSuccess;
  if (max_ny > TB) return hipErrorInvalidValue;
  // widest column block whose LDS (2*max_ny + TB entries per column) fits in 64 KiB
  const size_t per_col = sizeof(typename cvec<T>::type) * (2 * (size_t)max_ny + TB);
  const size_t cap = 65536;
  if (q >= 8 && 8 * per_col <= cap) return launch_solve_qb<T, 8>(op, leaves, nleaf, max_ny, q, G, rhs, x, s);
  if (q >= 4 && 4 * per_col <= cap) return launch_solve_qb<T, 4>(op, leaves, nleaf, max_ny, q, G, rhs, x, s);
  if (q >= 2 && 2 * per_col <= cap) return launch_solve_qb<T, 2>(op, leaves, nleaf, max_ny, q, G, rhs, x, s);
  return launch_solve_qb<T, 1>(op, leaves, nleaf, max_ny, q, G, rhs, x, s);
}

template hipError_t launch_leaf_solve<double>(const OpDev&, const BoxDev*, int, int, int, const c128*,
                                              const c128*, c128*, hipStream_t);
template hipError_t launch_leaf_solve<float>(const OpDev&, const BoxDev*, int, int, int, const c64*,
                                             const c128*, c128*, hipStream_t);
