// Two-ended block factorisation of the leaf box matrices A~_i (the local
// impedance problems of eq. (sub1)).
//
// The box matrix in line-major order (line j = all nodes with p = p0 + j, the
// ny nodes of a line contiguous) is block tridiagonal: the diagonal blocks
// are tridiagonal, the couplings between neighbouring lines are diagonal.
// With m = nx / 2 the factor keeps one inverse Schur complement per line,
// eliminated from both ends towards the middle line:
//   j < m   S_0 = A_00,        S_j = A_jj - A_{j,j-1} S_{j-1}^{-1} A_{j-1,j},  G_j = S_j^{-1}
//   j > m   T_{nx-1} = A_{..}, T_j = A_jj - A_{j,j+1} T_{j+1}^{-1} A_{j+1,j},  G_j = T_j^{-1}
//   j = m   G_m = (A_mm - A_{m,m-1} G_{m-1} A_{m-1,m} - A_{m,m+1} G_{m+1} A_{m+1,m})^{-1}.
// The two chains are independent work-groups; the middle line is a second
// launch.  G_j is stored column-major (b x b, b = ny) at goff + j b^2; the
// solve sweeps are in k_sweep.hip.
#include "dense.h"
#include "gj_reg.h"
#include "kernels.h"

namespace {

__device__ __forceinline__ double2 diag_block(const OpDev& op, const BoxDev& B, int j, int i, int k) {
  const int p = B.p0 + j, q = B.q0 + i;
  if (i == k) return stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, q, 0, 0);
  if (op.dim == 2 && (k == i + 1 || k == i - 1)) return stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, q, 0, k - i);
  return mk(0.0, 0.0);
}

// Lines handled by a work-group: the chain of one half (mode 0, block = 2 t
// + half) or the middle line (mode 1, block = t) of leaf lidx[t].  A line's
// Schur complement subtracts the eliminated neighbours nb[0..nnb).  info slot
// of the work-group: 2 leaf + half (mode 0) or leaf (mode 1).
struct LinePlan {
  int leaf, count, first, step, slot;
};

__device__ __forceinline__ LinePlan line_plan(const BoxDev* leaves, const int* lidx, int mode) {
  LinePlan P;
  if (mode == 0) {
    P.leaf = lidx[blockIdx.x >> 1];
    const int half = blockIdx.x & 1;
    P.slot = 2 * P.leaf + half;
    const int nx = leaves[P.leaf].nx, m = nx >> 1;
    P.count = half ? nx - 1 - m : m;
    P.first = half ? nx - 1 : 0;
    P.step = half ? -1 : 1;
  } else {
    P.leaf = lidx[blockIdx.x];
    P.slot = P.leaf;
    P.count = 1;
    P.first = leaves[P.leaf].nx >> 1;
    P.step = 1;
  }
  return P;
}

// neighbours already eliminated when line j is reached
__device__ __forceinline__ int eliminated(const BoxDev& B, int mode, int s, int j, int step, int (&nb)[2]) {
  if (mode == 0) {
    if (s == 0) return 0;
    nb[0] = j - step;
    return 1;
  }
  int n = 0;
  if (j >= 1) nb[n++] = j - 1;
  if (j + 1 < B.nx) nb[n++] = j + 1;
  return n;
}

// Global-memory variant for wide boxes: S_j is formed in place of G_j and
// inverted by the work-group with Gauss-Jordan elimination and partial
// pivoting, by panels of FNB pivots held in shared memory (512 threads).
constexpr int TBF = 512;
constexpr int FNB = 16;

size_t factor_shm(int b) { return sizeof(double2) * (2 * FNB * b + b + 2 * FNB) + sizeof(int) * (2 * b + FNB); }
__global__ void __launch_bounds__(TBF) k_leaf_factor(const OpDev* __restrict__ ops, const BoxDev* __restrict__ leaves,
                                                     const int* __restrict__ lidx, int mode,
                                                     c128* __restrict__ G, int* __restrict__ info) {
  const LinePlan P = line_plan(leaves, lidx, mode);
  const BoxDev B = leaves[P.leaf];
  const OpDev op = ops[B.prob];
  const int b = B.ny;
  const int tid = threadIdx.x;
  // typed double2 so that the dynamic block starts 16-byte aligned after the
  // static variables (misaligned 16-byte LDS accesses are split)
  extern __shared__ double2 smem_d2[];
  double2* work = smem_d2;                               // 2 FNB b
  double2* fcol = work + 2 * FNB * b;                    // b
  double2* rowk = fcol + b;                              // FNB
  double2* rold = rowk + FNB;                            // FNB
  int* src = reinterpret_cast<int*>(rold + FNB);         // b
  int* tot = src + b;                                    // b
  int* perm = tot + b;                                   // FNB
  __shared__ int s_piv;
  __shared__ int s_any;
  __shared__ int s_flag;
  if (tid == 0) s_flag = 0;
  int first = 0;
  // element (i, k) of this thread's first slot and the stride between slots
  const int i0 = tid % b, k0 = tid / b, di = TBF % b, dk = TBF / b;
  for (int s = 0; s < P.count; ++s) {
    const int j = P.first + P.step * s;
    c128* Gj = G + B.goff + (long long)j * b * b;
    int nb[2];
    const int nnb = eliminated(B, mode, s, j, P.step, nb);
    int i = i0, k = k0;
    while (k < b) {
      const long long e = i + (long long)k * b;
      double2 v = diag_block(op, B, j, i, k);
      for (int t = 0; t < nnb; ++t) {
        const c128* Gp = G + B.goff + (long long)nb[t] * b * b;
        const double2 ai = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j, B.q0 + i, nb[t] - j, 0);
        const double2 ak = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + nb[t], B.q0 + k, j - nb[t], 0);
        v = csub(v, cmul(cmul(ai, Gp[e]), ak));
      }
      Gj[e] = v;
      i += di;
      k += dk;
      if (i >= b) {
        i -= b;
        k += 1;
      }
    }
    __syncthreads();
    const int flag_before = s_flag;
    gj_inverse_blocked<TBF, FNB>(Gj, b, work, fcol, rowk, rold, src, tot, perm, &s_piv, &s_any, &s_flag);
    if (tid == 0 && first == 0 && flag_before == 0 && s_flag != 0) first = j * b + s_flag;
    __syncthreads();
  }
  if (tid == 0 && info) info[P.slot] = first;
}

// The same factorisation with S_j held in the registers of an NT-thread
// work-group and inverted there (thread: one row, columns strided by NT / b);
// G_j goes to memory once per line and is read back (cache-resident) to form
// the next line's Schur complement.
template <int NT, int RE>
__global__ void __launch_bounds__(NT) k_leaf_factor_reg(const OpDev* __restrict__ ops, const BoxDev* __restrict__ leaves,
                                                    const int* __restrict__ lidx, int mode,
                                                       c128* __restrict__ G, int* __restrict__ info) {
  const LinePlan P = line_plan(leaves, lidx, mode);
  const BoxDev B = leaves[P.leaf];
  const OpDev op = ops[B.prob];
  const int b = B.ny, nn = b * b;
  const int tid = threadIdx.x;
  __shared__ gjr::Scratch sc;
  if (tid == 0) sc.flag = 0;
  __syncthreads();
  const gjr::Layout L = gjr::layout<NT>(b);
  int first = 0;
  double2 A[RE];
  for (int s = 0; s < P.count; ++s) {
    const int j = P.first + P.step * s;
    c128* Gj = G + B.goff + (long long)j * nn;
    int nb[2];
    const int nnb = eliminated(B, mode, s, j, P.step, nb);
    // S_j; diagonal pivots first, row interchanges if they fail.  The line
    // couplings are real: a(i) G(i, k) a(k) with a = -(cells at the node's q
    // edges) / (2 h^2)
    const double ai = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + j, B.q0 + L.i, 1, 0).x;
    for (int attempt = 0; attempt < 2; ++attempt) {
#pragma unroll
      for (int r = 0; r < RE; ++r) {
        const int k = L.g + L.G * r;
        A[r] = (L.act && k < b) ? diag_block(op, B, j, L.i, k) : mk(0.0, 0.0);
      }
      for (int t = 0; t < nnb; ++t) {
        const c128* Gp = G + B.goff + (long long)nb[t] * nn;
#pragma unroll
        for (int r = 0; r < RE; ++r) {
          const int k = L.g + L.G * r;
          if (L.act && k < b) {
            const double ak = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + nb[t], B.q0 + k, 1, 0).x;
            A[r] = csub(A[r], cscale(Gp[L.i + (long long)k * b], ai * ak));
          }
        }
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
  if (tid == 0 && info) info[P.slot] = first;
}

template <int NT, int RE>
hipError_t launch_reg(const OpDev* ops, const BoxDev* leaves, int nleaf, const int* lidx, int count, c128* G,
                      int* info, hipStream_t s) {
  hipLaunchKernelGGL((k_leaf_factor_reg<NT, RE>), dim3(2 * count), dim3(NT), 0, s, ops, leaves, lidx, 0, G, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_leaf_factor_reg<NT, RE>), dim3(count), dim3(NT), 0, s, ops, leaves, lidx, 1, G,
                     info ? info + 2 * nleaf : nullptr);
  return hipGetLastError();
}

}  // namespace

// Register-slot class of a leaf of width ny (the kernel variant that holds
// its rows: 1024 threads, at most 4 or 6 entries per thread; 6: the
// global-memory variant).  The chains are few and sequential, so the widest
// work-group that holds the matrix hides the most latency per pivot step.
int leaf_factor_bucket(int ny) {
  if (ny > 256) return 6;
  const int G = 1024 / ny;
  const int re = G > 0 ? (ny + G - 1) / G : 1 << 30;
  if (re <= 4) return 0;
  if (re <= 6) return 1;
  return 6;  // wider rows would spill the register tile: the global-memory variant
}

// info: 3 nleaf ints (two chains per leaf, then the middle lines); nonzero =
// (line * b + pivot step + 1) of the first zero pivot.  Factors the count
// leaves lidx[0 .. count) (of nleaf), whose widths are at most max_ny.
hipError_t launch_leaf_factor(const OpDev* ops, const BoxDev* leaves, int nleaf, const int* lidx, int count,
                              int max_ny, c128* G, int* info, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  switch (leaf_factor_bucket(max_ny)) {
    case 0: return launch_reg<1024, 4>(ops, leaves, nleaf, lidx, count, G, info, s);
    case 1: return launch_reg<1024, 6>(ops, leaves, nleaf, lidx, count, G, info, s);
    default: break;
  }
  if (max_ny > 256) return hipErrorInvalidValue;
  const size_t shm = factor_shm(max_ny);
  // the limit is raised once, to what the widest leaf needs: setting it per launch
  // would let a concurrent set-up (another thread) lower it between another
  // launch's setting and that launch
  static const hipError_t raised = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&k_leaf_factor), hipFuncAttributeMaxDynamicSharedMemorySize, (int)factor_shm(256));
  if (shm > 65536 && raised != hipSuccess) return raised;
  hipLaunchKernelGGL(k_leaf_factor, dim3(2 * count), dim3(TBF), shm, s, ops, leaves, lidx, 0, G, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_leaf_factor, dim3(count), dim3(TBF), shm, s, ops, leaves, lidx, 1, G,
                     info ? info + 2 * nleaf : nullptr);
  return hipGetLastError();
}
