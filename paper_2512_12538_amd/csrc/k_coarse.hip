// Coarse space of one level: the Galerkin matrix A_c = C^H A C and its
// inverse (eq. (coarse1)), and the per-iteration coarse correction
// u += C A_c^{-1} C^H t.  C = (C_i) has disjoint supports (the owned boxes of
// the restricted prolongation), so C^H t and C y are independent per box and
// A_c is block-sparse: block (i, j) is non-zero only when the owned box of i
// meets the owned box of j dilated by the 5-point stencil.
#include "kernels.h"

namespace {

constexpr int TB = 256;
constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ bool owns(const BoxDev& B, int p, int q) {
  return p >= B.op0 && p <= B.op1 && q >= B.oq0 && q <= B.oq1;
}

// AC[box][b][x] = (A_P C_box[b])(x) for x in the dilated owned box dil = (p0, p1, q0, q1)
__global__ void __launch_bounds__(TB) k_galerkin_ac(OpDev op, const BoxDev* __restrict__ boxes,
                                                    const BoxDev* __restrict__ par, const int4* __restrict__ dil,
                                                    int rmax, const c128* __restrict__ C, c128* __restrict__ AC) {
  const int box = blockIdx.y / rmax, col = blockIdx.y % rmax;
  const BoxDev B = boxes[box];
  if (col >= B.r) return;
  const BoxDev P = par[B.parent];
  const int4 d = dil[box];
  const int dny = d.w - d.z + 1;
  const int nd = (d.y - d.x + 1) * dny;
  const c128* c = C + B.coff + (long long)col * B.n_own;
  c128* out = AC + B.acoff + (long long)col * nd;
  const int DP[5] = {0, -1, 1, 0, 0};
  const int DQ[5] = {0, 0, 0, -1, 1};
  for (int t = blockIdx.x * TB + threadIdx.x; t < nd; t += gridDim.x * TB) {
    const int xp = d.x + t / dny, xq = d.z + t % dny;
    double2 acc = mk(0.0, 0.0);
    for (int k = 0; k < 5; ++k) {
      if (op.dim == 1 && k >= 3) break;
      const int yp = xp + DP[k], yq = xq + DQ[k];
      if (yp < P.p0 || yp > P.p1 || yq < P.q0 || yq > P.q1) continue;
      if (!owns(B, yp, yq)) continue;
      const double2 a = stencil_coef(op, P.p0, P.p1, P.q0, P.q1, xp, xq, DP[k], DQ[k]);
      acc = cfma(a, c[(long long)(yp - B.op0) * B.own_ny + (yq - B.oq0)], acc);
    }
    out[t] = acc;
  }
}

// A_c[cidx_i + a][cidx_j + b] = sum over own_i cap dil_j of conj(C_i[a]) AC_j[b];
// block (pair, a), one wave per b.
__global__ void __launch_bounds__(TB) k_galerkin_blocks(const BoxDev* __restrict__ boxes,
                                                        const ParentDev* __restrict__ pars,
                                                        const int4* __restrict__ pairs, int rmax,
                                                        const int4* __restrict__ dil, const c128* __restrict__ C,
                                                        const c128* __restrict__ AC, c128* __restrict__ Ac) {
  const int pr = blockIdx.x / rmax, a = blockIdx.x % rmax;
  const int4 pp = pairs[pr];  // (i, j, parent, -)
  const BoxDev Bi = boxes[pp.x], Bj = boxes[pp.y];
  if (a >= Bi.r) return;
  const ParentDev P = pars[pp.z];
  const int4 d = dil[pp.y];
  const int dny = d.w - d.z + 1;
  const int nd = (d.y - d.x + 1) * dny;
  const int lo_p = max(Bi.op0, d.x), hi_p = min(Bi.op1, d.y);
  const int lo_q = max(Bi.oq0, d.z), hi_q = min(Bi.oq1, d.w);
  const int np = hi_p - lo_p + 1, nq = hi_q - lo_q + 1;
  const int cnt = (np > 0 && nq > 0) ? np * nq : 0;
  const c128* ci = C + Bi.coff + (long long)a * Bi.n_own;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  for (int b = wv; b < Bj.r; b += TB / WAVE) {
    const c128* acj = AC + Bj.acoff + (long long)b * nd;
    double2 acc = mk(0.0, 0.0);
    for (int t = lane; t < cnt; t += WAVE) {
      const int xp = lo_p + t / nq, xq = lo_q + t % nq;
      const double2 u = ci[(long long)(xp - Bi.op0) * Bi.own_ny + (xq - Bi.oq0)];
      const double2 v = acj[(long long)(xp - d.x) * dny + (xq - d.z)];
      acc = cfmac(u, v, acc);
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (lane == 0) Ac[P.aoff + (long long)(Bj.cidx + b) * P.n_c + (Bi.cidx + a)] = acc;
  }
}

// Gauss-Jordan inversion of every parent's A_c spread over the whole GPU: one
// launch per pivot selects and interchanges the pivot row, scales it and saves
// the pivot column; a second launch eliminates the column from all other rows
// with one thread per matrix entry.
__global__ void __launch_bounds__(TB) k_gj_pivot(const ParentDev* __restrict__ pars, c128* __restrict__ Aall,
                                                 int* __restrict__ perm_all, c128* __restrict__ fcol_all, int max_nc,
                                                 int kk, int* __restrict__ info) {
  const ParentDev P = pars[blockIdx.x];
  const int n = P.n_c;
  if (kk >= n) return;
  c128* A = Aall + P.aoff;
  int* perm = perm_all + (long long)blockIdx.x * max_nc;
  c128* fcol = fcol_all + (long long)blockIdx.x * max_nc;
  const int tid = threadIdx.x;
  __shared__ double rv[TB];
  __shared__ int ri[TB];
  double best = -1.0;
  int bi = kk;
  for (int i = kk + tid; i < n; i += TB) {
    const double a = cabs2(A[i + (long long)kk * n]);
    if (a > best) { best = a; bi = i; }
  }
  rv[tid] = best;
  ri[tid] = bi;
  __syncthreads();
  for (int st = TB / 2; st > 0; st >>= 1) {
    if (tid < st) {
      const double o = rv[tid + st];
      const int oi = ri[tid + st];
      if (o > rv[tid] || (o == rv[tid] && oi < ri[tid])) { rv[tid] = o; ri[tid] = oi; }
    }
    __syncthreads();
  }
  const int pr = ri[0];
  if (tid == 0) {
    perm[kk] = pr;
    if (rv[0] <= 0.0 && info[blockIdx.x] == 0) info[blockIdx.x] = kk + 1;
  }
  if (pr != kk) {
    for (int c = tid; c < n; c += TB) {
      const double2 t = A[kk + (long long)c * n];
      A[kk + (long long)c * n] = A[pr + (long long)c * n];
      A[pr + (long long)c * n] = t;
    }
  }
  __syncthreads();
  const double2 pv = A[kk + (long long)kk * n];
  const double2 inv = cabs2(pv) > 0.0 ? cdiv(mk(1.0, 0.0), pv) : mk(0.0, 0.0);
  for (int i = tid; i < n; i += TB) fcol[i] = (i == kk) ? mk(0.0, 0.0) : A[i + (long long)kk * n];
  __syncthreads();
  for (int c = tid; c < n; c += TB) {
    const long long e = kk + (long long)c * n;
    A[e] = (c == kk) ? inv : cmul(A[e], inv);
  }
}

__global__ void __launch_bounds__(TB) k_gj_elim(const ParentDev* __restrict__ pars, c128* __restrict__ Aall,
                                                const c128* __restrict__ fcol_all, int max_nc, int kk) {
  const ParentDev P = pars[blockIdx.y];
  const int n = P.n_c;
  if (kk >= n) return;
  c128* A = Aall + P.aoff;
  const c128* fcol = fcol_all + (long long)blockIdx.y * max_nc;
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)TB + threadIdx.x; e < nn; e += (long long)gridDim.x * TB) {
    const int i = (int)(e % n), c = (int)(e / n);
    if (i == kk) continue;
    const double2 base = (c == kk) ? mk(0.0, 0.0) : A[e];
    A[e] = csub(base, cmul(fcol[i], A[kk + (long long)c * n]));
  }
}

// undo the row interchanges as column interchanges (last first), one row per thread
__global__ void __launch_bounds__(TB) k_gj_unperm(const ParentDev* __restrict__ pars, c128* __restrict__ Aall,
                                                  const int* __restrict__ perm_all, int max_nc) {
  const ParentDev P = pars[blockIdx.y];
  const int n = P.n_c;
  c128* A = Aall + P.aoff;
  const int* perm = perm_all + (long long)blockIdx.y * max_nc;
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  for (int kk = n - 1; kk >= 0; --kk) {
    const int pk = perm[kk];
    if (pk != kk) {
      const double2 t = A[i + (long long)kk * n];
      A[i + (long long)kk * n] = A[i + (long long)pk * n];
      A[i + (long long)pk * n] = t;
    }
  }
}

// cvec[par][b][cidx + k] = C_child[k]^H t[par][b][owned nodes of child];
// block (child, group of KC columns, chunk of QC right-hand sides), so C is
// read q/QC times and t r/KC times.
constexpr int KC = 4, QC = 8;

__global__ void __launch_bounds__(TB) k_coarse_restrict(const BoxDev* __restrict__ child,
                                                        const BoxDev* __restrict__ par,
                                                        const ParentDev* __restrict__ pd, int kgroups, int q,
                                                        const c128* __restrict__ C, const c128* __restrict__ t,
                                                        c128* __restrict__ cvec) {
  const int box = blockIdx.x / kgroups, k0 = (blockIdx.x % kgroups) * KC;
  const int b0 = blockIdx.y * QC;
  const BoxDev B = child[box];
  if (k0 >= B.r) return;
  const BoxDev P = par[B.parent];
  const ParentDev D = pd[B.parent];
  double2 acc[KC][QC];
#pragma unroll
  for (int a = 0; a < KC; ++a)
#pragma unroll
    for (int c = 0; c < QC; ++c) acc[a][c] = mk(0.0, 0.0);
  for (int e = threadIdx.x; e < B.n_own; e += TB) {
    const int oa = e / B.own_ny, oc = e - oa * B.own_ny;
    const long long pl = (long long)(B.op0 + oa - P.p0) * P.ny + (B.oq0 + oc - P.q0);
    double2 cv[KC];
#pragma unroll
    for (int a = 0; a < KC; ++a)
      cv[a] = k0 + a < B.r ? C[B.coff + (long long)(k0 + a) * B.n_own + e] : mk(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < QC; ++c) {
      if (b0 + c < q) {
        const double2 tv = t[P.voff * q + (long long)(b0 + c) * P.n + pl];
#pragma unroll
        for (int a = 0; a < KC; ++a) acc[a][c] = cfmac(cv[a], tv, acc[a][c]);
      }
    }
  }
  __shared__ double sx[TB], sy[TB];
#pragma unroll
  for (int a = 0; a < KC; ++a)
#pragma unroll
    for (int c = 0; c < QC; ++c) {
      sx[threadIdx.x] = acc[a][c].x;
      sy[threadIdx.x] = acc[a][c].y;
      __syncthreads();
      for (int st = TB / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
          sx[threadIdx.x] += sx[threadIdx.x + st];
          sy[threadIdx.x] += sy[threadIdx.x + st];
        }
        __syncthreads();
      }
      if (threadIdx.x == 0 && k0 + a < B.r && b0 + c < q)
        cvec[D.yoff * q + (long long)(b0 + c) * D.n_c + B.cidx + k0 + a] = mk(sx[0], sy[0]);
      __syncthreads();
    }
}

// y[par][b] = A_c^{-1} cvec[par][b]: block (64 rows, parent, rhs), four column
// slices per row reduced in LDS.
__global__ void __launch_bounds__(TB) k_coarse_gemv(const ParentDev* __restrict__ pd, int q,
                                                    const c128* __restrict__ Ainv, const c128* __restrict__ cvec,
                                                    c128* __restrict__ y) {
  const int pb = blockIdx.y / q, col = blockIdx.y % q;
  const ParentDev D = pd[pb];
  const int n = D.n_c;
  const int r0 = blockIdx.x * 64;
  if (r0 >= n) return;
  const c128* cv = cvec + D.yoff * q + (long long)col * n;
  const c128* A = Ainv + D.aoff;
  const int rr = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int r = r0 + rr;
  double2 acc = mk(0.0, 0.0);
  if (r < n)
    for (int c = sl; c < n; c += 4) acc = cfma(A[r + (long long)c * n], cv[c], acc);
  __shared__ double2 red[4][64];
  red[sl][rr] = acc;
  __syncthreads();
  if (sl == 0 && r < n) {
    const double2 s = cadd(cadd(red[0][rr], red[1][rr]), cadd(red[2][rr], red[3][rr]));
    y[D.yoff * q + (long long)col * n + r] = s;
  }
}

// u[par][b][owned nodes of child] += C_child y: one thread per owned node, QC
// right-hand sides per thread so C is read q/QC times.
__global__ void __launch_bounds__(TB) k_coarse_prolong(const BoxDev* __restrict__ child,
                                                       const BoxDev* __restrict__ par,
                                                       const ParentDev* __restrict__ pd, int q,
                                                       const c128* __restrict__ C, const c128* __restrict__ y,
                                                       c128* __restrict__ u) {
  const int box = blockIdx.y;
  const int b0 = blockIdx.z * QC;
  const BoxDev B = child[box];
  if (B.r == 0) return;
  const BoxDev P = par[B.parent];
  const ParentDev D = pd[B.parent];
  __shared__ double2 ys[QC][128];
  for (int e = threadIdx.x; e < QC * B.r; e += TB) {
    const int c = e / B.r, k = e % B.r;
    ys[c][k] = b0 + c < q ? y[D.yoff * q + (long long)(b0 + c) * D.n_c + B.cidx + k] : mk(0.0, 0.0);
  }
  __syncthreads();
  for (int e = blockIdx.x * TB + threadIdx.x; e < B.n_own; e += gridDim.x * TB) {
    double2 acc[QC];
#pragma unroll
    for (int c = 0; c < QC; ++c) acc[c] = mk(0.0, 0.0);
    for (int k = 0; k < B.r; ++k) {
      const double2 cv = C[B.coff + (long long)k * B.n_own + e];
#pragma unroll
      for (int c = 0; c < QC; ++c) acc[c] = cfma(cv, ys[c][k], acc[c]);
    }
    const int oa = e / B.own_ny, oc = e - oa * B.own_ny;
    const long long pl = (long long)(B.op0 + oa - P.p0) * P.ny + (B.oq0 + oc - P.q0);
#pragma unroll
    for (int c = 0; c < QC; ++c) {
      if (b0 + c < q) {
        c128* uv = u + P.voff * q + (long long)(b0 + c) * P.n;
        uv[pl] = cadd(uv[pl], acc[c]);
      }
    }
  }
}

inline int gx(long long n, int cap) {
  long long g = (n + TB - 1) / TB;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_galerkin_ac(const OpDev& op, const BoxDev* boxes, int nbox, const BoxDev* par, const int4* dil,
                              int max_dil, int rmax, const c128* C, c128* AC, hipStream_t s) {
  if (nbox <= 0 || rmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_galerkin_ac, dim3(gx(max_dil, 256), nbox * rmax), dim3(TB), 0, s, op, boxes, par, dil, rmax,
                     C, AC);
  return hipGetLastError();
}

hipError_t launch_galerkin_blocks(const BoxDev* boxes, const ParentDev* pars, const int4* pairs, int npairs,
                                  int rmax, const int4* dil, const c128* C, const c128* AC, c128* Ac,
                                  hipStream_t s) {
  if (npairs <= 0 || rmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_galerkin_blocks, dim3(npairs * rmax), dim3(TB), 0, s, boxes, pars, pairs, rmax, dil, C, AC,
                     Ac);
  return hipGetLastError();
}

hipError_t launch_gj_inverse(const ParentDev* pars, int npar, int max_nc, c128* A, int* piv, c128* fcol, int* info,
                             hipStream_t s) {
  if (npar <= 0 || max_nc <= 0) return hipSuccess;
  hipError_t e = launch_fill_zero(info, (long long)sizeof(int) * npar, s);
  if (e != hipSuccess) return e;
  const long long nn = (long long)max_nc * max_nc;
  const int gxe = gx(nn, 1024);
  for (int kk = 0; kk < max_nc; ++kk) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(npar), dim3(TB), 0, s, pars, A, piv, fcol, max_nc, kk, info);
    hipLaunchKernelGGL(k_gj_elim, dim3(gxe, npar), dim3(TB), 0, s, pars, A, fcol, max_nc, kk);
  }
  hipLaunchKernelGGL(k_gj_unperm, dim3((max_nc + TB - 1) / TB, npar), dim3(TB), 0, s, pars, A, piv, max_nc);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict(const BoxDev* child, int nchild, const BoxDev* par, const ParentDev* pd,
                                  int rmax, int q, const c128* C, const c128* t, c128* cvec, hipStream_t s) {
  if (nchild <= 0 || rmax <= 0 || q <= 0) return hipSuccess;
  const int kgroups = (rmax + KC - 1) / KC;
  hipLaunchKernelGGL(k_coarse_restrict, dim3(nchild * kgroups, (q + QC - 1) / QC), dim3(TB), 0, s, child, par, pd,
                     kgroups, q, C, t, cvec);
  return hipGetLastError();
}

hipError_t launch_coarse_gemv(const ParentDev* pd, int npar, int max_nc, int q, const c128* Ainv,
                              const c128* cvec, c128* y, hipStream_t s) {
  if (npar <= 0 || max_nc <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_gemv, dim3((max_nc + 63) / 64, npar * q), dim3(TB), 0, s, pd, q, Ainv, cvec, y);
  return hipGetLastError();
}

hipError_t launch_coarse_prolong(const BoxDev* child, int nchild, int max_own, const BoxDev* par,
                                 const ParentDev* pd, int q, const c128* C, const c128* y, c128* u,
                                 hipStream_t s) {
  if (nchild <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_prolong, dim3(gx(max_own, 256), nchild, (q + QC - 1) / QC), dim3(TB), 0, s, child,
                     par, pd, q, C, y, u);
  return hipGetLastError();
}
