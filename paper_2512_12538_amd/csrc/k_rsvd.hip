// Interface map T_i and the randomised SVD of Sec. 2:
//   sample    Y = T_i Omega = B_i^o S_i(B_i^T Omega),  B_ij = B_j A~_j R_j P_i,
//   orthogonalise  Q = qr(Y),
//   adjoint   B^H = T_i^* Q = B_i conj(S_i(conj((B_i^o)^H Q))),
//   small SVD of B, V_i = dominant right singular vectors,
//   extension C_i = P_i S_i(B_i^T V_i).
// Here: the interface scatter/gather, the trace to the neighbours and its
// adjoint (stencil rows evaluated on the fly), a batched Householder QR, a
// one-sided Jacobi SVD and the small products between them.
#include "kernels.h"

namespace {

constexpr int TB = 256;
constexpr int TBS = 1024;  // the small dense factorisations: one item (column, column pair) per wave
constexpr int WAVE = 64;

// Sum over the 64 lanes, returned in every lane, without LDS: DPP within each
// row of 16 (lane ^ 1, lane ^ 2, rotations by 4 and 8), then the gfx950
// permlane16 / permlane32 swaps across rows and halves; the lanes add in
// different orders, so the first lane's sum is broadcast and every lane holds
// the same bits.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp<0xb1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp<0x4e>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp<0x124>(v);  // row_ror:4
  v += dpp<0x128>(v);  // row_ror:8
  {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false,
                                                     false);
    v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false,
                                                     false);
    v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  }
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ __forceinline__ double2 wave_sum(double2 v) { return mk(wave_sum(v.x), wave_sum(v.y)); }

__global__ void __launch_bounds__(TB) k_iface_scatter(const BoxDev* __restrict__ boxes, int q,
                                                      const int* __restrict__ if_idx,
                                                      const long long* __restrict__ voffs,
                                                      const c128* __restrict__ vals, int use_r,
                                                      c128* __restrict__ buf) {
  const int box = blockIdx.y / q, col = blockIdx.y % q;
  const BoxDev B = boxes[box];
  const int ncol = use_r ? B.r : B.s;
  if (col >= ncol) return;
  const long long base = B.voff * q + (long long)col * B.n;
  const c128* v = vals + voffs[box] + (long long)col * B.m_in;
  for (int t = blockIdx.x * TB + threadIdx.x; t < B.m_in; t += gridDim.x * TB)
    buf[base + if_idx[B.if_off + t]] = v[t];
}

__global__ void __launch_bounds__(TB) k_iface_gather(const BoxDev* __restrict__ boxes, int q,
                                                     const int* __restrict__ if_idx,
                                                     const long long* __restrict__ voffs,
                                                     const c128* __restrict__ buf, c128* __restrict__ vals,
                                                     int use_r, int conj_in) {
  const int box = blockIdx.y / q, col = blockIdx.y % q;
  const BoxDev B = boxes[box];
  const int ncol = use_r ? B.r : B.s;
  if (col >= ncol) return;
  const long long base = B.voff * q + (long long)col * B.n;
  c128* v = vals + voffs[box] + (long long)col * B.m_in;
  for (int t = blockIdx.x * TB + threadIdx.x; t < B.m_in; t += gridDim.x * TB) {
    const double2 x = buf[base + if_idx[B.if_off + t]];
    v[t] = conj_in ? cconj(x) : x;
  }
}

__device__ __forceinline__ bool owns(const BoxDev& B, int p, int q) {
  return p >= B.op0 && p <= B.op1 && q >= B.oq0 && q <= B.oq1;
}

// Y[box][col][row] = sum over the stencil of row x of box j of
// A~_j[x, y] (P_i X)[y]  (only owned nodes y of box i contribute).
__global__ void __launch_bounds__(TB) k_trace(const OpDev* __restrict__ ops, const BoxDev* __restrict__ boxes, int q,
                                              const int2* __restrict__ rows, const long long* __restrict__ yoff,
                                              const c128* __restrict__ X, c128* __restrict__ Y) {
  const int box = blockIdx.y / q, col = blockIdx.y % q;
  const BoxDev Bi = boxes[box];
  if (col >= Bi.s) return;
  const OpDev op = ops[Bi.prob];  // siblings share the problem
  const long long xb = Bi.voff * q + (long long)col * Bi.n;
  c128* y = Y + yoff[box] + (long long)col * Bi.tr_cnt;
  for (int r = blockIdx.x * TB + threadIdx.x; r < Bi.tr_cnt; r += gridDim.x * TB) {
    const int2 rw = rows[Bi.tr_off + r];
    const BoxDev Bj = boxes[rw.x];
    const int xp = Bj.p0 + rw.y / Bj.ny, xq = Bj.q0 + rw.y % Bj.ny;
    double2 acc = mk(0.0, 0.0);
    const int DP[5] = {0, -1, 1, 0, 0};
    const int DQ[5] = {0, 0, 0, -1, 1};
    for (int d = 0; d < 5; ++d) {
      if (op.dim == 1 && d >= 3) break;
      const int yp = xp + DP[d], yq = xq + DQ[d];
      if (yp < Bj.p0 || yp > Bj.p1 || yq < Bj.q0 || yq > Bj.q1) continue;
      if (!owns(Bi, yp, yq)) continue;
      const double2 a = stencil_coef(op, Bj.p0, Bj.p1, Bj.q0, Bj.q1, xp, xq, DP[d], DQ[d]);
      acc = cfma(a, X[xb + (long long)(yp - Bi.p0) * Bi.ny + (yq - Bi.q0)], acc);
    }
    y[r] = acc;
  }
}

// H[box][col][y] = conj of the sum over trace rows (j, x) reaching y of
// conj(A~_j[x, y]) Q[row][col], i.e. sum A~_j[x, y] conj(Q[row][col]): the
// conjugated adjoint trace that the solve of B^H = B_i conj(S_i(conj(.))) takes
// (the conjugations are exact, so writing it conjugated saves a pass)
__global__ void __launch_bounds__(TB) k_trace_adjoint(const OpDev* __restrict__ ops, const BoxDev* __restrict__ boxes, int q,
                                                      const int2* __restrict__ rows,
                                                      const int* __restrict__ seg_ptr,
                                                      const int* __restrict__ seg_y,
                                                      const int4* __restrict__ adj,
                                                      const long long* __restrict__ yoff,
                                                      const c128* __restrict__ Qm, c128* __restrict__ H) {
  const int box = blockIdx.y / q, col = blockIdx.y % q;
  const BoxDev Bi = boxes[box];
  if (col >= Bi.s) return;
  const long long hb = Bi.voff * q + (long long)col * Bi.n;
  const c128* qv = Qm + yoff[box] + (long long)col * Bi.tr_cnt;
  for (int sg = blockIdx.x * TB + threadIdx.x; sg < Bi.adj_cnt; sg += gridDim.x * TB) {
    const int s = Bi.adj_off + sg;
    double2 acc = mk(0.0, 0.0);
    for (int e = seg_ptr[s]; e < seg_ptr[s + 1]; ++e) {
      const int4 a = adj[e];  // (row, dp, dq, -)
      const int2 rw = rows[Bi.tr_off + a.x];
      const BoxDev Bj = boxes[rw.x];
      const int xp = Bj.p0 + rw.y / Bj.ny, xq = Bj.q0 + rw.y % Bj.ny;
      const double2 c = stencil_coef(ops[Bj.prob], Bj.p0, Bj.p1, Bj.q0, Bj.q1, xp, xq, a.y, a.z);
      acc = cfmac(c, qv[a.x], acc);
    }
    H[hb + seg_y[s]] = cconj(acc);
  }
}

// Batched Householder QR, one work-group per problem.  On exit A holds the
// explicit thin Q (columns >= min(m, n) are zero) and R the n x n upper factor.
__global__ void __launch_bounds__(TBS) k_qr(const int* __restrict__ ms, const int* __restrict__ ns,
                                           const long long* __restrict__ aoff, c128* __restrict__ Aall,
                                           const long long* __restrict__ roff, c128* __restrict__ Rall,
                                           c128* __restrict__ Wall) {
  const int pb = blockIdx.x;
  const int m = ms[pb], n = ns[pb];
  c128* A = Aall + aoff[pb];
  c128* Vr = Wall + aoff[pb];  // reflectors, same shape as A
  c128* R = Rall + roff[pb];
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE, nw = TBS / WAVE;
  __shared__ double s_tau[128];
  __shared__ double2 s_alpha;
  const int kq = m < n ? m : n;
  for (int e = tid; e < n * n; e += TBS) R[e] = mk(0.0, 0.0);
  for (int k = 0; k < kq; ++k) {
    if (wv == 0) {
      double nrm2 = 0.0;
      for (int i = k + lane; i < m; i += WAVE) nrm2 += cabs2(A[i + (long long)k * m]);
      nrm2 = wave_sum(nrm2);
      const double2 x0 = A[k + (long long)k * m];
      const double ax0 = sqrt(cabs2(x0));
      const double nrm = sqrt(nrm2);
      double2 alpha = ax0 > 0.0 ? mk(-x0.x / ax0 * nrm, -x0.y / ax0 * nrm) : mk(-nrm, 0.0);
      const double2 v0 = csub(x0, alpha);
      const double vn2 = nrm2 - ax0 * ax0 + cabs2(v0);
      for (int i = lane; i < m; i += WAVE) {
        double2 v = mk(0.0, 0.0);
        if (i == k) v = v0;
        else if (i > k) v = A[i + (long long)k * m];
        Vr[i + (long long)k * m] = v;
      }
      if (lane == 0) {
        s_tau[k] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        if (nrm2 == 0.0) alpha = mk(0.0, 0.0);
        s_alpha = alpha;
      }
    }
    __syncthreads();
    const double tau = s_tau[k];
    if (tid == 0) R[k + (long long)k * n] = s_alpha;
    for (int c = k + 1 + wv; c < n; c += nw) {
      double2 d = mk(0.0, 0.0);
      for (int i = k + lane; i < m; i += WAVE) d = cfmac(Vr[i + (long long)k * m], A[i + (long long)c * m], d);
      d = wave_sum(d);
      const double2 f = cscale(d, tau);
      for (int i = k + lane; i < m; i += WAVE) {
        const long long e = i + (long long)c * m;
        A[e] = csub(A[e], cmul(f, Vr[i + (long long)k * m]));
      }
    }
    __syncthreads();
    for (int c = k + 1 + tid; c < n; c += TBS) R[k + (long long)c * n] = A[k + (long long)c * m];
    __syncthreads();
  }
  // explicit Q = H_0 H_1 ... H_{kq-1} [I; 0]
  for (int e = tid; e < m * n; e += TBS) {
    const int i = e % m, c = e / m;
    A[e] = (i == c && c < kq) ? mk(1.0, 0.0) : mk(0.0, 0.0);
  }
  __syncthreads();
  for (int k = kq - 1; k >= 0; --k) {
    const double tau = s_tau[k];
    for (int c = k + wv; c < kq; c += nw) {
      double2 d = mk(0.0, 0.0);
      for (int i = k + lane; i < m; i += WAVE) d = cfmac(Vr[i + (long long)k * m], A[i + (long long)c * m], d);
      d = wave_sum(d);
      const double2 f = cscale(d, tau);
      for (int i = k + lane; i < m; i += WAVE) {
        const long long e = i + (long long)c * m;
        A[e] = csub(A[e], cmul(f, Vr[i + (long long)k * m]));
      }
    }
    __syncthreads();
  }
}

// One-sided (Hestenes) Jacobi on the columns of R (n x n), round-robin pair
// order, one wave per pair.  Output: U[:, t] = columns of R J normalised and
// sorted by decreasing norm (the left singular vectors of R), sigma sorted.
// INLDS: R is copied to shared memory (dynamic, n_max^2 entries) and rotated
// there; R in memory is left as it was.
template <bool INLDS>
__global__ void __launch_bounds__(TBS) k_jacobi(const int* __restrict__ ns, const long long* __restrict__ roff,
                                               c128* __restrict__ Rall, const long long* __restrict__ uoff,
                                               c128* __restrict__ Uall, double* __restrict__ sig,
                                               const long long* __restrict__ soff) {
  const int pb = blockIdx.x;
  const int n = ns[pb];
  extern __shared__ double2 rlds[];
  c128* R = Rall + roff[pb];
  if constexpr (INLDS) {
    for (int e = threadIdx.x; e < n * n; e += TBS) rlds[e] = R[e];
    __syncthreads();
    R = rlds;
  }
  c128* U = Uall + uoff[pb];
  double* sg = sig + soff[pb];
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE, nw = TBS / WAVE;
  __shared__ int s_rot;
  __shared__ double s_norm[128];
  __shared__ int s_ord[128];
  const int N2 = n + (n & 1);
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < N2 - 1; ++rnd) {
      for (int pk = wv; pk < N2 / 2; pk += nw) {
        int a, b;
        if (pk == 0) { a = rnd; b = N2 - 1; }
        else { a = (rnd + pk) % (N2 - 1); b = (rnd - pk + N2 - 1) % (N2 - 1); }
        if (a >= n || b >= n) continue;
        const int p = a < b ? a : b, qq = a < b ? b : a;
        double al = 0.0, be = 0.0;
        double2 ga = mk(0.0, 0.0);
        for (int i = lane; i < n; i += WAVE) {
          const double2 x = R[i + (long long)p * n], y = R[i + (long long)qq * n];
          al += cabs2(x);
          be += cabs2(y);
          ga = cfmac(x, y, ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        const double ag = sqrt(cabs2(ga));
        if (ag > tol * sqrt(al * be) && ag > 0.0) {
          const double zeta = (be - al) / (2.0 * ag);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          const double2 ph = mk(ga.x / ag, -ga.y / ag);  // e^{-i phi}
          for (int i = lane; i < n; i += WAVE) {
            const double2 x = R[i + (long long)p * n];
            const double2 y = cmul(ph, R[i + (long long)qq * n]);
            R[i + (long long)p * n] = mk(c * x.x - s * y.x, c * x.y - s * y.y);
            R[i + (long long)qq * n] = mk(s * x.x + c * y.x, s * x.y + c * y.y);
          }
          if (lane == 0) s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) break;
  }
  for (int c = wv; c < n; c += nw) {
    double a = 0.0;
    for (int i = lane; i < n; i += WAVE) a += cabs2(R[i + (long long)c * n]);
    a = wave_sum(a);
    if (lane == 0) s_norm[c] = sqrt(a);
  }
  __syncthreads();
  if (tid == 0) {
    for (int c = 0; c < n; ++c) s_ord[c] = c;
    for (int x = 0; x < n; ++x) {
      int best = x;
      for (int y = x + 1; y < n; ++y)
        if (s_norm[s_ord[y]] > s_norm[s_ord[best]]) best = y;
      int t = s_ord[x]; s_ord[x] = s_ord[best]; s_ord[best] = t;
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += TBS) {
    const int i = e % n, c = e / n;
    const int src = s_ord[c];
    const double nv = s_norm[src];
    U[e] = nv > 0.0 ? cscale(R[i + (long long)src * n], 1.0 / nv) : mk(0.0, 0.0);
  }
  for (int c = tid; c < n; c += TBS) sg[c] = s_norm[s_ord[c]];
}

__global__ void __launch_bounds__(TB) k_small_gemm(const int* __restrict__ ms, const int* __restrict__ ns,
                                                   const int* __restrict__ rs, const long long* __restrict__ qoff,
                                                   const c128* __restrict__ Q, const long long* __restrict__ uoff,
                                                   const c128* __restrict__ U, const long long* __restrict__ voff,
                                                   c128* __restrict__ V) {
  const int pb = blockIdx.y;
  const int m = ms[pb], n = ns[pb], r = rs[pb];
  const c128* Qp = Q + qoff[pb];
  const c128* Up = U + uoff[pb];
  c128* Vp = V + voff[pb];
  for (int e = blockIdx.x * TB + threadIdx.x; e < m * r; e += gridDim.x * TB) {
    const int i = e % m, c = e / m;
    double2 acc = mk(0.0, 0.0);
    for (int k = 0; k < n; ++k) acc = cfma(Qp[i + (long long)k * m], Up[k + (long long)c * n], acc);
    Vp[e] = acc;
  }
}

__global__ void __launch_bounds__(TB) k_extract_owned(const BoxDev* __restrict__ boxes, int q,
                                                      const c128* __restrict__ buf, c128* __restrict__ C) {
  const int box = blockIdx.y / q, col = blockIdx.y % q;
  const BoxDev B = boxes[box];
  if (col >= B.r) return;
  const long long base = B.voff * q + (long long)col * B.n;
  c128* c = C + B.coff + (long long)col * B.n_own;
  for (int t = blockIdx.x * TB + threadIdx.x; t < B.n_own; t += gridDim.x * TB) {
    const int oa = t / B.own_ny, oc = t - oa * B.own_ny;
    c[t] = buf[base + (long long)(B.op0 + oa - B.p0) * B.ny + (B.oq0 + oc - B.q0)];
  }
}

inline int gx(long long n, int cap = 256) {
  long long g = (n + TB - 1) / TB;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_iface_scatter(const BoxDev* boxes, int nbox, int q, const int* if_idx, const long long* voff,
                                const c128* vals, int use_r, c128* buf, hipStream_t s) {
  if (nbox <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iface_scatter, dim3(4, nbox * q), dim3(TB), 0, s, boxes, q, if_idx, voff, vals, use_r, buf);
  return hipGetLastError();
}

hipError_t launch_iface_gather(const BoxDev* boxes, int nbox, int q, const int* if_idx, const long long* voff,
                               const c128* buf, c128* vals, int use_r, int conj_in, hipStream_t s) {
  if (nbox <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iface_gather, dim3(4, nbox * q), dim3(TB), 0, s, boxes, q, if_idx, voff, buf, vals, use_r,
                     conj_in);
  return hipGetLastError();
}

hipError_t launch_trace(const OpDev* ops, const BoxDev* boxes, int nbox, int q, const int2* rows,
                        const long long* yoff, const c128* X, c128* Y, hipStream_t s) {
  if (nbox <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace, dim3(8, nbox * q), dim3(TB), 0, s, ops, boxes, q, rows, yoff, X, Y);
  return hipGetLastError();
}

hipError_t launch_trace_adjoint(const OpDev* ops, const BoxDev* boxes, int nbox, int q, const int2* rows,
                                const int* seg_ptr, const int* seg_y, const int4* adj, const long long* yoff,
                                const c128* Qm, c128* H, hipStream_t s) {
  if (nbox <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace_adjoint, dim3(8, nbox * q), dim3(TB), 0, s, ops, boxes, q, rows, seg_ptr, seg_y,
                     adj, yoff, Qm, H);
  return hipGetLastError();
}

hipError_t launch_qr(int nprob, const int* m, const int* n, const long long* aoff, c128* A, const long long* roff,
                     c128* R, c128* work, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qr, dim3(nprob), dim3(TBS), 0, s, m, n, aoff, A, roff, R, work);
  return hipGetLastError();
}

namespace {
constexpr int kJacobiLds = 96;  // 96^2 complex128 = 144 KiB of shared memory
// raised once, to the largest matrix kept in shared memory (a per-call setting
// could be lowered by a concurrent caller before another's launch)
hipError_t jacobi_lds_limit() {
  static const hipError_t raised = hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi<true>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)(sizeof(double2) * kJacobiLds * kJacobiLds));
  return raised;
}
}  // namespace

hipError_t launch_jacobi_svd(int nprob, const int* n, int nmax, const long long* roff, c128* R, const long long* uoff,
                             c128* U, double* sigma, const long long* soff, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  const size_t shm = sizeof(double2) * (size_t)nmax * nmax;
  if (nmax <= kJacobiLds && (shm <= 65536 || jacobi_lds_limit() == hipSuccess))
    hipLaunchKernelGGL(k_jacobi<true>, dim3(nprob), dim3(TBS), shm, s, n, roff, R, uoff, U, sigma, soff);
  else
    hipLaunchKernelGGL(k_jacobi<false>, dim3(nprob), dim3(TBS), 0, s, n, roff, R, uoff, U, sigma, soff);
  return hipGetLastError();
}

hipError_t launch_small_gemm(int nprob, int max_mr, const int* m, const int* n, const int* r, const long long* qoff,
                             const c128* Q, const long long* uoff, const c128* U, const long long* voff, c128* V,
                             hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_gemm, dim3(gx(max_mr, 64), nprob), dim3(TB), 0, s, m, n, r, qoff, Q, uoff, U, voff, V);
  return hipGetLastError();
}

hipError_t launch_extract_owned(const BoxDev* boxes, int nbox, int max_own, int q, const c128* buf, c128* C,
                                hipStream_t s) {
  if (nbox <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_extract_owned, dim3(gx(max_own, 64), nbox * q), dim3(TB), 0, s, boxes, q, buf, C);
  return hipGetLastError();
}
