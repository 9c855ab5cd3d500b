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
#include "gj_reg.h"
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

// The same block LU with the Schur complement S_j held in the registers of an
// NT-thread work-group and inverted there (thread: one row, columns strided
// by NT / b); G_j goes to memory once per line and is read back
// (cache-resident) to form S_{j+1}.
template <int NT, int RE>
__global__ void __launch_bounds__(NT) k_leaf_factor_reg(OpDev op, const BoxDev* __restrict__ leaves,
                                                       c128* __restrict__ G, int* __restrict__ info) {
  const BoxDev B = leaves[blockIdx.x];
  const int b = B.ny, nn = b * b;
  const int tid = threadIdx.x;
  __shared__ gjr::Scratch sc;
  if (tid == 0) sc.flag = 0;
  __syncthreads();
  const gjr::Layout L = gjr::layout<NT>(b);
  int first = 0;
  double2 A[RE];
  const double2 ai = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + 1, B.q0 + L.i, -1, 0);
  for (int j = 0; j < B.nx; ++j) {
    c128* Gj = G + B.goff + (long long)j * nn;
    const c128* Gp = Gj - nn;
    // S_j = A_jj - A_{j,j-1} G_{j-1} A_{j-1,j}; diagonal pivots first, row interchanges if they fail
    for (int attempt = 0; attempt < 2; ++attempt) {
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int k = L.g + L.G * r;
        double2 v = mk(0.0, 0.0);
        if (L.act && k < b) {
          v = diag_block(op, B, j, L.i, k);
          if (j > 0) {
            const double2 ak = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j - 1, B.q0 + k, 1, 0);
            v = csub(v, cmul(cmul(ai, Gp[L.i + (long long)k * b]), ak));
          }
        }
        A[r] = v;
      }
      if (attempt == 0) {
        if (gjr::invert_diag<NT, RE>(A, b, L, sc, 0.25)) break;
      } else {
        gjr::invert<NT, RE>(A, b, L, sc);
      }
    }
    if (first == 0 && sc.flag != 0) first = j * b + sc.flag;
    if (L.act) {
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int c = L.g + L.G * r;
        if (c < b) Gj[L.i + (long long)sc.pos[c] * b] = A[r];
      }
    }
    __syncthreads();
    if (tid == 0) sc.flag = 0;
    __syncthreads();
  }
  if (tid == 0 && info) info[blockIdx.x] = first;
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

// Pipelined sweeps: the same recurrence with the next line's G_j slice (and
// the next line's right-hand side) loaded into registers while the current
// one is applied (G does not depend on the data, only the short y_j chain
// does).  Threads exchange data through LDS only, so the barriers order LDS
// alone and the prefetches stay in flight across them: two barriers per line,
// the reduction of line j fused with the construction of y_{j+1}.  Thread
// (kap, i) holds G_j[k][i] for k = kap + K r, r < R.  Work-groups of one leaf
// are placed on one XCD (dispatch is round-robin over the 8 XCDs) so the
// column chunks of a leaf share that XCD's L2 copy of G.
template <typename T, int QB, int R, int NTP>
__global__ void __launch_bounds__(NTP) k_leaf_solve_pipe(OpDev op, const BoxDev* __restrict__ leaves, int nleaf,
                                                        int nchunk, int q, const typename cvec<T>::type* __restrict__ G,
                                                        const c128* __restrict__ rhs, c128* __restrict__ x) {
  typedef typename cvec<T>::type CT;
  int leaf, chunk;
  if ((nleaf & 7) == 0) {
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    leaf = xcd + 8 * (slot / nchunk);
    chunk = slot % nchunk;
  } else {
    leaf = blockIdx.x / nchunk;
    chunk = blockIdx.x % nchunk;
  }
  const BoxDev B = leaves[leaf];
  const int b = B.ny;
  int K = NTP / b;
  if (K > b) K = b;
  const int YP = K * R;  // rows of y (padded): entries k >= b stay zero; y[k*QB + c]
  const int tid = threadIdx.x;
  const int kap = tid / b, i = tid - kap * b;
  const bool act = kap < K;
  const int kc = act ? kap : K - 1;  // idle threads shadow a valid slice and discard the result
  const int c0 = chunk * QB;
  __shared__ CT y[QB * 256];
  __shared__ CT part[QB * NTP];
  const long long base = B.voff * q;
  const long long bb = (long long)b * b;
  const CT* Gl = G + B.goff;
  // this thread's slice: rows k = kc*R + r; reads past b land in padding and are masked
  const int kbase = kc * R;
  const int goff0 = kbase * b + i;
  // reduction slots of this thread: e = tid + NTP t < b*QB (b <= NTP, so t < QB)
  int eii[QB], ecol[QB];
  bool eok[QB];
#pragma unroll
  for (int t = 0; t < QB; ++t) {
    const int e = tid + NTP * t;
    eii[t] = e % b;
    ecol[t] = e / b;
    eok[t] = e < b * QB && (c0 + ecol[t] < q);
  }
  CT g[R];  // G_j slice; each entry is reloaded with G_{j+-1} right after its last use
  double2 pre[QB];
  const CT zero = mk((T)0, (T)0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const CT v = Gl[goff0 + b * r];
    g[r] = (kbase + r < b) ? v : zero;
  }
  for (int e = tid; e < QB * YP; e += NTP) y[e] = zero;
  lds_barrier();
  // y_0 = b_0
  for (int e = tid; e < b * QB; e += NTP) {
    const int k = e % b, c = e / b;
    y[k * QB + c] = (c0 + c < q) ? from_c128<T>(rhs[base + (long long)(c0 + c) * B.n + k]) : zero;
  }
  lds_barrier();
  // ---------------- forward: w_j = G_j y_j, y_{j+1} = b_{j+1} - A_{j+1,j} w_j
  for (int j = 0; j < B.nx; ++j) {
    const int jn = j + 1 < B.nx ? j + 1 : B.nx - 2;  // the backward sweep starts at G_{nx-2}
    const CT* Gn = Gl + (long long)jn * bb;
    const int jr = j + 1 < B.nx ? j + 1 : j;
#pragma unroll
    for (int t = 0; t < QB; ++t) {
      const int cc = eok[t] ? c0 + ecol[t] : 0;
      pre[t] = rhs[base + (long long)cc * B.n + (long long)jr * b + eii[t]];
    }
    CT acc[QB];
#pragma unroll
    for (int c = 0; c < QB; ++c) acc[c] = zero;
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < QB; ++c) acc[c] = cfma(g[r], y[(kbase + r) * QB + c], acc[c]);
      const CT v = Gn[goff0 + b * r];
      g[r] = (kbase + r < b) ? v : zero;
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < QB; ++c) part[(kap * QB + c) * b + i] = acc[c];
    }
    lds_barrier();
#pragma unroll
    for (int t = 0; t < QB; ++t) {
      const int e = tid + NTP * t;
      if (e < b * QB) {
        const int ii = eii[t], c = ecol[t];
        CT sacc = part[c * b + ii];
        for (int kp = 1; kp < K; ++kp) sacc = cadd(sacc, part[(kp * QB + c) * b + ii]);
        const double2 w = to_c128(sacc);
        if (eok[t]) x[base + (long long)(c0 + c) * B.n + (long long)j * b + ii] = w;
        double2 yn;
        if (j + 1 < B.nx) {
          const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j + 1, B.q0 + ii, -1, 0);
          yn = eok[t] ? csub(pre[t], cmul(a, w)) : mk(0.0, 0.0);
        } else {
          // start of the backward sweep: y = A_{nx-2,nx-1} x_{nx-1}
          const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j - 1, B.q0 + ii, 1, 0);
          yn = cmul(a, w);
        }
        y[ii * QB + c] = from_c128<T>(yn);
      }
    }
    lds_barrier();
  }
  // ---------------- backward: x_j = w_j - G_j A_{j,j+1} x_{j+1}
  for (int j = B.nx - 2; j >= 0; --j) {
    const int jn = j > 0 ? j - 1 : 0;
    const CT* Gn = Gl + (long long)jn * bb;
#pragma unroll
    for (int t = 0; t < QB; ++t) {
      const int cc = eok[t] ? c0 + ecol[t] : 0;
      pre[t] = x[base + (long long)cc * B.n + (long long)j * b + eii[t]];
    }
    CT acc[QB];
#pragma unroll
    for (int c = 0; c < QB; ++c) acc[c] = zero;
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < QB; ++c) acc[c] = cfma(g[r], y[(kbase + r) * QB + c], acc[c]);
      const CT v = Gn[goff0 + b * r];
      g[r] = (kbase + r < b) ? v : zero;
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < QB; ++c) part[(kap * QB + c) * b + i] = acc[c];
    }
    lds_barrier();
#pragma unroll
    for (int t = 0; t < QB; ++t) {
      const int e = tid + NTP * t;
      if (e < b * QB) {
        const int ii = eii[t], c = ecol[t];
        CT sacc = part[c * b + ii];
        for (int kp = 1; kp < K; ++kp) sacc = cadd(sacc, part[(kp * QB + c) * b + ii]);
        double2 xv = mk(0.0, 0.0);
        if (eok[t]) {
          xv = csub(pre[t], to_c128(sacc));
          x[base + (long long)(c0 + c) * B.n + (long long)j * b + ii] = xv;
        }
        if (j > 0) {
          const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j - 1, B.q0 + ii, 1, 0);
          y[ii * QB + c] = from_c128<T>(cmul(a, xv));
        }
      }
    }
    lds_barrier();
  }
}

template <typename T, int QB, int R, int NTP>
hipError_t launch_pipe(const OpDev& op, const BoxDev* leaves, int nleaf, int q, const typename cvec<T>::type* G,
                       const c128* rhs, c128* x, hipStream_t s) {
  const int nchunk = (q + QB - 1) / QB;
  hipLaunchKernelGGL((k_leaf_solve_pipe<T, QB, R, NTP>), dim3(nleaf * nchunk), dim3(NTP), 0, s, op, leaves, nleaf,
                     nchunk, q, G, rhs, x);
  return hipGetLastError();
}

// Launch rule measured on MI355X for the 4x4 / N=256 leaves (b = 67..69):
// complex128 prefers one right-hand side per work-group of 512 threads for
// small batches (the L2 serves the shared G_j) and four per 256-thread
// work-group for large ones; complex64 four per 512-thread work-group.
// Configurations whose register tile would spill are never chosen.
template <typename T>
hipError_t launch_pipe_auto(const OpDev& op, const BoxDev* leaves, int nleaf, int max_ny, int q,
                            const typename cvec<T>::type* G, const c128* rhs, c128* x, hipStream_t s, bool& done) {
  done = true;
  auto kr = [&](int nt, int& K, int& R) {
    K = nt / max_ny;
    if (K > max_ny) K = max_ny;
    R = K > 0 ? (max_ny + K - 1) / K : 1 << 30;
  };
  int K256, R256, K512, R512;
  kr(256, K256, R256);
  kr(512, K512, R512);
  const bool fit256 = R256 <= 24 && K256 * 24 <= 256;
  const bool fit512 = R512 <= 12 && K512 * 12 <= 256;
  if (sizeof(typename cvec<T>::type) == 16) {
    if (q >= 48 && fit256) return launch_pipe<T, 4, 24, 256>(op, leaves, nleaf, q, G, rhs, x, s);
    if (fit512) return launch_pipe<T, 1, 12, 512>(op, leaves, nleaf, q, G, rhs, x, s);
    if (fit256) return launch_pipe<T, 1, 24, 256>(op, leaves, nleaf, q, G, rhs, x, s);
  } else {
    if (fit512) {
      if (q >= 32) return launch_pipe<T, 4, 12, 512>(op, leaves, nleaf, q, G, rhs, x, s);
      if (q >= 2) return launch_pipe<T, 2, 12, 512>(op, leaves, nleaf, q, G, rhs, x, s);
      return launch_pipe<T, 1, 12, 512>(op, leaves, nleaf, q, G, rhs, x, s);
    }
    if (fit256) {
      if (q >= 4) return launch_pipe<T, 4, 24, 256>(op, leaves, nleaf, q, G, rhs, x, s);
      return launch_pipe<T, 1, 24, 256>(op, leaves, nleaf, q, G, rhs, x, s);
    }
  }
  done = false;
  return hipSuccess;
}

}  // namespace

hipError_t launch_leaf_factor(const OpDev& op, const BoxDev* leaves, int nleaf, int max_ny, c128* G,
                              int* info, hipStream_t s) {
  if (nleaf <= 0) return hipSuccess;
  const long long nn = (long long)max_ny * max_ny;
  if (max_ny <= 256) {
    // one row per thread, columns strided by NT / b; a narrower box needs fewer slots
    const int G512 = 512 / max_ny;
    const int re = G512 > 0 ? (max_ny + G512 - 1) / G512 : 1 << 30;
    if (re <= 8) {
      hipLaunchKernelGGL((k_leaf_factor_reg<512, 8>), dim3(nleaf), dim3(512), 0, s, op, leaves, G, info);
      return hipGetLastError();
    }
    if (re <= 10) {
      hipLaunchKernelGGL((k_leaf_factor_reg<512, 10>), dim3(nleaf), dim3(512), 0, s, op, leaves, G, info);
      return hipGetLastError();
    }
    if (re <= 12) {
      hipLaunchKernelGGL((k_leaf_factor_reg<512, 12>), dim3(nleaf), dim3(512), 0, s, op, leaves, G, info);
      return hipGetLastError();
    }
    if (re <= 16) {
      hipLaunchKernelGGL((k_leaf_factor_reg<512, 16>), dim3(nleaf), dim3(512), 0, s, op, leaves, G, info);
      return hipGetLastError();
    }
    if (re <= 24) {
      hipLaunchKernelGGL((k_leaf_factor_reg<512, 24>), dim3(nleaf), dim3(512), 0, s, op, leaves, G, info);
      return hipGetLastError();
    }
    if (re <= 48) {
      hipLaunchKernelGGL((k_leaf_factor_reg<512, 48>), dim3(nleaf), dim3(512), 0, s, op, leaves, G, info);
      return hipGetLastError();
    }
  }
  const size_t shm = sizeof(double2) * max_ny + (sizeof(double) + sizeof(int)) * TB + sizeof(int) * max_ny;
  hipLaunchKernelGGL(k_leaf_factor, dim3(nleaf), dim3(TB), shm, s, op, leaves, G, info);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_leaf_solve(const OpDev& op, const BoxDev* leaves, int nleaf, int max_ny, int q,
                             const typename cvec<T>::type* G, const c128* rhs, c128* x, hipStream_t s) {
  if (nleaf <= 0 || q <= 0) return hipSuccess;
  if (max_ny > TB) return hipErrorInvalidValue;
  {
    bool done = false;
    const hipError_t e = launch_pipe_auto<T>(op, leaves, nleaf, max_ny, q, G, rhs, x, s, done);
    if (done) return e;
  }
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
