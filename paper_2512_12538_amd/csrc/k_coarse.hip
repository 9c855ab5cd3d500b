// Coarse space of one level: the Galerkin matrix A_c = C^H A C and its
// inverse (eq. (coarse1)), and the per-iteration coarse correction
// u += C A_c^{-1} C^H t.  C = (C_i) has disjoint supports (the owned boxes of
// the restricted prolongation), so C^H t and C y are independent per box and
// A_c is block-sparse: block (i, j) is non-zero only when the owned box of i
// meets the owned box of j dilated by the 5-point stencil.
#include <algorithm>

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
__global__ void __launch_bounds__(TB) k_galerkin_ac(const OpDev* __restrict__ ops, const BoxDev* __restrict__ boxes,
                                                    const BoxDev* __restrict__ par, const int4* __restrict__ dil,
                                                    int rmax, const c128* __restrict__ C, c128* __restrict__ AC) {
  const int box = blockIdx.y / rmax, col = blockIdx.y % rmax;
  const BoxDev B = boxes[box];
  const OpDev op = ops[B.prob];
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

// A mode t of box i whose column of C_i has a norm of at most tol times the
// box's largest column norm is dropped: the column is zeroed (so A_c gets a zero
// row and column there) and drop[i * rmax + t] = 1.  One work-group per box,
// one wave per column.
constexpr int TBD = 1024;
__global__ void __launch_bounds__(TBD) k_drop_negligible(const BoxDev* __restrict__ boxes, int rmax, double tol,
                                                         c128* __restrict__ C, int* __restrict__ drop) {
  const BoxDev B = boxes[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ double nrm[128];
  __shared__ double big;
  for (int t = threadIdx.x; t < rmax; t += TBD) drop[(long long)blockIdx.x * rmax + t] = 0;
  if (B.r == 0) return;
  c128* Cb = C + B.coff;
  for (int t = wv; t < B.r; t += TBD / 64) {
    double a = 0.0;
    for (int e = lane; e < B.n_own; e += 64) a += cabs2(Cb[(long long)t * B.n_own + e]);
    a = wave_sum(a);
    if (lane == 0) nrm[t] = sqrt(a);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int t = 0; t < B.r; ++t) mx = fmax(mx, nrm[t]);
    big = mx;
  }
  __syncthreads();
  const double lim = tol * big;
  for (int t = wv; t < B.r; t += TBD / 64) {
    if (nrm[t] > lim) continue;
    if (lane == 0) drop[(long long)blockIdx.x * rmax + t] = 1;
    for (int e = lane; e < B.n_own; e += 64) Cb[(long long)t * B.n_own + e] = mk(0.0, 0.0);
  }
}

// A_c[cidx + t][cidx + t] = 1 for the dropped modes (their row and column are
// zero), so the inverse gives them a zero coarse value.
__global__ void k_unit_dropped(const BoxDev* __restrict__ boxes, const ParentDev* __restrict__ pd, int nbox,
                               int rmax, const int* __restrict__ drop, c128* __restrict__ A) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbox * rmax) return;
  const int box = idx / rmax, t = idx - box * rmax;
  const BoxDev B = boxes[box];
  if (t >= B.r || !drop[idx]) return;
  const ParentDev D = pd[B.parent];
  const long long d = B.cidx + t;
  A[D.aoff + d + d * D.n_c] = mk(1.0, 0.0);
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

// ---- blocked Gauss-Jordan: panels of GJ_NB pivots.  k_gj_panel runs the
// panel's steps (partial pivoting, the same step as above) on the n x nb panel
// in shared memory, one work-group per parent, and writes the panel back (its
// columns then hold the panel's elimination matrix E restricted to them) with
// the panel's row permutation sig (new row i = old row sig[i]).  k_gj_trail
// applies the panel to every other column x: x <- S x + (E[:, K] - I[:, K]) (S x)_K,
// one work-group per (parent, column), the column staged in shared memory.
constexpr int GJ_NB = 16;
constexpr int GJ_MAXN = 512;

__global__ void __launch_bounds__(1024) k_gj_panel(const ParentDev* __restrict__ pars, c128* __restrict__ Aall,
                                                   int* __restrict__ perm_all, int* __restrict__ sig_all, int max_nc,
                                                   int k0, int* __restrict__ info) {
  const ParentDev P = pars[blockIdx.x];
  const int n = P.n_c;
  if (k0 >= n) return;
  const int kb = n - k0 < GJ_NB ? n - k0 : GJ_NB;
  c128* A = Aall + P.aoff;
  int* perm = perm_all + (long long)blockIdx.x * max_nc;
  int* sig = sig_all + (long long)blockIdx.x * max_nc;
  // shared: pan[t * n + i] (t < kb), fcol[n], rowk[GJ_NB], rold[GJ_NB], ssig[n]
  extern __shared__ double2 pan[];
  double2* fcol = pan + (long long)GJ_NB * n;
  double2* rowk = fcol + n;
  double2* rold = rowk + GJ_NB;
  int* ssig = reinterpret_cast<int*>(rold + GJ_NB);
  __shared__ int s_p, s_flag;
  const int tid = threadIdx.x, NT = blockDim.x;
  // element (i, c) of this thread's first slot and the stride between slots
  const int i0 = tid % n, c0 = tid / n, di = NT % n, dc = NT / n;
  {
    int i = i0, c = c0;
    while (c < kb) {
      pan[i + c * n] = A[i + (long long)(k0 + c) * n];
      i += di;
      c += dc;
      if (i >= n) { i -= n; c += 1; }
    }
  }
  for (int i = tid; i < n; i += NT) ssig[i] = i;
  if (tid == 0) s_flag = 0;
  __syncthreads();
  // two barriers a pivot: the first wave finds the pivot and stages the step
  // (scaled pivot row, old row kk, multipliers of the interchanged column),
  // then every thread updates the panel with the interchange folded in
  for (int t = 0; t < kb; ++t) {
    const int kk = k0 + t;
    const double2* col = pan + (long long)t * n;
    if (tid < 64) {
      double best = -1.0;
      int p = kk;
      for (int i = kk + tid; i < n; i += 64) {
        const double a = cabs2(col[i]);
        if (a > best) { best = a; p = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(p, o, 64);
        if (ob > best || (ob == best && oi < p)) { best = ob; p = oi; }
      }
      const double2 pv = col[p];
      const double2 inv = cabs2(pv) > 0.0 ? cdiv(mk(1.0, 0.0), pv) : mk(0.0, 0.0);
      for (int c = tid; c < kb; c += 64) {
        rold[c] = pan[(long long)c * n + kk];
        rowk[c] = (c == t) ? inv : cmul(pan[(long long)c * n + p], inv);
      }
      for (int i = tid; i < n; i += 64) fcol[i] = (i == kk) ? mk(0.0, 0.0) : (i == p ? col[kk] : col[i]);
      if (tid == 0) {
        s_p = p;
        perm[kk] = p;
        if (best <= 0.0 && s_flag == 0) s_flag = kk + 1;
        const int tmp = ssig[kk];
        ssig[kk] = ssig[p];
        ssig[p] = tmp;
      }
    }
    __syncthreads();
    const int p = s_p;
    int i = i0, c = c0;
    while (c < kb) {
      const int e = i + c * n;
      if (i == kk) {
        pan[e] = rowk[c];
      } else {
        const double2 base = (c == t) ? mk(0.0, 0.0) : (i == p ? rold[c] : pan[e]);
        pan[e] = csub(base, cmul(fcol[i], rowk[c]));
      }
      i += di;
      c += dc;
      if (i >= n) { i -= n; c += 1; }
    }
    __syncthreads();
  }
  {
    int i = i0, c = c0;
    while (c < kb) {
      A[i + (long long)(k0 + c) * n] = pan[i + c * n];
      i += di;
      c += dc;
      if (i >= n) { i -= n; c += 1; }
    }
  }
  for (int i = tid; i < n; i += NT) sig[i] = ssig[i];
  if (tid == 0 && s_flag != 0 && info[blockIdx.x] == 0) info[blockIdx.x] = s_flag;
}

__global__ void __launch_bounds__(256) k_gj_trail(const ParentDev* __restrict__ pars, c128* __restrict__ Aall,
                                                  const int* __restrict__ sig_all, int max_nc, int k0) {
  const ParentDev P = pars[blockIdx.y];
  const int n = P.n_c, c = blockIdx.x;
  if (k0 >= n || c >= n) return;
  const int kb = n - k0 < GJ_NB ? n - k0 : GJ_NB;
  if (c >= k0 && c < k0 + kb) return;
  c128* A = Aall + P.aoff;
  const int* sig = sig_all + (long long)blockIdx.y * max_nc;
  __shared__ double2 xs[GJ_MAXN];
  __shared__ double2 xk[GJ_NB];
  c128* xc = A + (long long)c * n;
  for (int i = threadIdx.x; i < n; i += 256) xs[i] = xc[sig[i]];
  __syncthreads();
  if (threadIdx.x < kb) xk[threadIdx.x] = xs[k0 + threadIdx.x];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    double2 v = xs[i];
    for (int t = 0; t < kb; ++t) {
      double2 w = A[i + (long long)(k0 + t) * n];
      if (i == k0 + t) w = csub(w, mk(1.0, 0.0));
      v = cfma(w, xk[t], v);
    }
    xc[i] = v;
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

// ---- the coarse products as FP64 matrix-core (MFMA 16x16x4) products.
// Operand layouts of v_mfma_f64_16x16x4f64 (one wave): lane l holds
// A[l & 15][l >> 4] and B[l >> 4][l & 15]; D[4 s + (l >> 4)][l & 15] is slot s
// of lane l.  A complex product takes four real products on (re, im) parts.
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// (re, im) += a * b
__device__ __forceinline__ void cmfma(double2 a, double2 b, d4& re, d4& im) {
  re = mfma(a.x, b.x, re);
  re = mfma(-a.y, b.y, re);
  im = mfma(a.x, b.y, im);
  im = mfma(a.y, b.x, im);
}
// (re, im) += conj(a) * b
__device__ __forceinline__ void cmfma_ca(double2 a, double2 b, d4& re, d4& im) {
  re = mfma(a.x, b.x, re);
  re = mfma(a.y, b.y, re);
  im = mfma(a.x, b.y, im);
  im = mfma(-a.y, b.x, im);
}

// parent-local index of owned node e of child B
__device__ __forceinline__ long long owned_to_parent(const BoxDev& B, const BoxDev& P, int e) {
  const int oa = e / B.own_ny, oc = e - oa * B.own_ny;
  return (long long)(B.op0 + oa - P.p0) * P.ny + (B.oq0 + oc - P.q0);
}

constexpr int RCH = 128;  // owned nodes per restrict work-group (split of the inner dimension)
constexpr int RST = 17;   // LDS row stride (double2) of a staged C column slice of 16 nodes

// LDS written by some lanes of a wave and read by others: a wave's LDS
// operations complete in issue order, so fences and a compiler barrier suffice
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}
constexpr int KU = 8;     // inner steps whose operands are loaded before their products

// Restriction work items: chunk g = (child, chunk index) of RCH owned nodes,
// the chunks of all children with a coarse space numbered consecutively
// (child order), column group cg = 16 right-hand sides.  One wave per
// (g, cg), items cg-fastest: with many right-hand sides the four waves of a
// work-group share a chunk (and its C loads), with few they take consecutive
// chunks.  part[g][a][c] = sum over the chunk's owned nodes e of conj(C[e][a])
// t[c][e] (a < 16 MT, c < 16 ncg).  Operands of KU steps of four nodes are
// loaded before their products, so KU (1 + MT) loads per lane are in flight.
// A wave's arithmetic does not depend on which items share its work-group.
// Only the q real right-hand-side columns of a tile are written; with active
// flags (problem * q + column) a wave none of whose columns is active returns
// at once (the columns it owns belong to converged systems only).
template <int MT>
__global__ void __launch_bounds__(TB) k_restrict_mfma(const BoxDev* __restrict__ child, const BoxDev* __restrict__ par,
                                                      const int2* __restrict__ chunks, int nitems, int ncg, int q,
                                                      const c128* __restrict__ C, const c128* __restrict__ t,
                                                      c128* __restrict__ part, const int* __restrict__ active) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int item = blockIdx.x * (TB / 64) + wave;
  if (item >= nitems) return;
  const int g = item / ncg, cg = item - g * ncg;
  const int2 bc = chunks[g];
  const BoxDev B = child[bc.x];
  if (active) {
    // a wave whose right-hand sides are all converged leaves its tile as it is
    bool any = false;
    for (int cc = cg * 16; cc < q && cc < cg * 16 + 16; ++cc) any = any || active[B.prob * q + cc];
    if (!any) return;
  }
  const int e0 = bc.y * RCH;
  const BoxDev P = par[B.parent];
  const int m = lane & 15, kk = lane >> 4;
  const int c = cg * 16 + m;
  const int e1 = e0 + RCH < B.n_own ? e0 + RCH : B.n_own;
  const c128* tb = t + P.voff * q + (long long)(c < q ? c : 0) * P.n;
  const c128* Cb = C + B.coff;
  constexpr int U = MT <= 2 ? KU : MT <= 4 ? KU / 2 : KU / 4;  // loads in flight within the register budget
  d4 re[MT], im[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) re[mt] = im[mt] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = e0; k0 < e1; k0 += 4 * U) {
    double2 tv[U], cv[U][MT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = k0 + 4 * u + kk;
      const bool ve = e < e1;
      tv[u] = (ve && c < q) ? tb[owned_to_parent(B, P, e)] : mk(0.0, 0.0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int a = mt * 16 + m;
        cv[u][mt] = (ve && a < B.r) ? Cb[(long long)a * B.n_own + e] : mk(0.0, 0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        if (mt * 16 < B.r) cmfma_ca(cv[u][mt], tv[u], re[mt], im[mt]);  // tiles past this box's rank skipped
  }
  const int qpad = ncg * 16;
  c128* pb = part + (long long)g * (MT * 16) * qpad;
  if (c < q) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        const int a = mt * 16 + 4 * sl + (lane >> 4);
        pb[(long long)a * qpad + c] = mk(re[mt][sl], im[mt][sl]);
      }
  }
}

// cvec[par][c][cidx + a] = sum over the child's chunks of part[g][a][c];
// cbase[child] = its first chunk.  Work-group: RS_OUT outputs (a, c) of one
// child x RS_SEG chains; chain k sums the chunks k, k + RS_SEG, ... in turn,
// then one thread per output adds the RS_SEG chain sums in chain order.  The
// order depends on the child's chunk count only (not on q): a box with
// thousands of chunks is summed by 64 chains in parallel instead of one.
constexpr int RS_SEG = 64, RS_OUT = 16;
__global__ void __launch_bounds__(RS_SEG * RS_OUT) k_restrict_sum(const BoxDev* __restrict__ child,
                                                                  const ParentDev* __restrict__ pd,
                                                                  const int* __restrict__ cbase, int rpad, int q,
                                                                  int qpad, const c128* __restrict__ part,
                                                                  c128* __restrict__ cvec) {
  const int box = blockIdx.y;
  const BoxDev B = child[box];
  if (blockIdx.x * RS_OUT >= B.r * q) return;  // the same for the whole work-group
  const int o = threadIdx.x % RS_OUT, sg = threadIdx.x / RS_OUT;
  const int idx = blockIdx.x * RS_OUT + o;
  const int a = idx / q, c = idx - a * q;
  const bool live = a < B.r;
  const int nch = (B.n_own + RCH - 1) / RCH;
  const long long st = (long long)rpad * qpad;
  double2 acc = mk(0.0, 0.0);
  if (live) {
    const c128* pb = part + (long long)cbase[box] * st + (long long)a * qpad + c;
    // eight loads in flight, added in chunk order
    constexpr int RU = 8;
    int ch = sg;
    for (; ch + (RU - 1) * RS_SEG < nch; ch += RU * RS_SEG) {
      double2 v[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) v[u] = pb[(ch + u * RS_SEG) * st];
#pragma unroll
      for (int u = 0; u < RU; ++u) acc = cadd(acc, v[u]);
    }
    for (; ch < nch; ch += RS_SEG) acc = cadd(acc, pb[ch * st]);
  }
  __shared__ double2 red[RS_SEG][RS_OUT];
  red[sg][o] = acc;
  __syncthreads();
  if (sg == 0 && live) {
    double2 sum = red[0][o];
    for (int k = 1; k < RS_SEG; ++k) sum = cadd(sum, red[k][o]);
    const ParentDev D = pd[B.parent];
    cvec[D.yoff * q + (long long)c * D.n_c + B.cidx + a] = sum;
  }
}

// y[par][c] = A_c^{-1} cvec[par][c]: one work-group per 16 x 16 output tile
// (rows of A_c^{-1} x right-hand sides); its four waves take interleaved
// quarters of the inner dimension (KU steps of four at a time) and meet in LDS.
__global__ void __launch_bounds__(TB) k_coarse_gemm(const ParentDev* __restrict__ pd, int q, int ntiles,
                                                    const c128* __restrict__ Ainv, const c128* __restrict__ cvec,
                                                    c128* __restrict__ y) {
  const ParentDev D = pd[blockIdx.y];
  const int n = D.n_c;
  const int mt = blockIdx.x / ntiles, nt = blockIdx.x - mt * ntiles;
  if (mt * 16 >= n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, kk = lane >> 4;
  const int row = mt * 16 + m, col = nt * 16 + m;
  const c128* A = Ainv + D.aoff;
  const c128* cv = cvec + D.yoff * q;
  d4 re = {0.0, 0.0, 0.0, 0.0}, im = re;
  for (int k0 = wave * 4 * KU; k0 < n; k0 += 4 * 4 * KU) {
    double2 av[KU], bv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = k0 + 4 * u + kk;
      av[u] = (row < n && k < n) ? A[row + (long long)k * n] : mk(0.0, 0.0);
      bv[u] = (k < n && col < q) ? cv[(long long)col * n + k] : mk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) cmfma(av[u], bv[u], re, im);
  }
  __shared__ double2 red[4][256];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) red[wave][sl * 64 + lane] = mk(re[sl], im[sl]);
  __syncthreads();
  if (wave == 0) {
    const int cc = nt * 16 + (lane & 15);
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const double2 v = cadd(cadd(red[0][sl * 64 + lane], red[1][sl * 64 + lane]),
                             cadd(red[2][sl * 64 + lane], red[3][sl * 64 + lane]));
      const int r = mt * 16 + 4 * sl + (lane >> 4);
      if (r < n && cc < q) y[D.yoff * q + (long long)cc * n + r] = v;
    }
  }
}

// u[par][c][owned nodes of child] += C_child y: computed transposed,
// (y^T C^T)[c][e], so that a wave's D tile spans 16 consecutive owned nodes.
// Wave: 16 nodes x 16 NTL right-hand sides (NTL tiles); inner dimension r.
// The box's y block (r x 16 NTL) is staged in LDS once per box; each lane
// loads its C column slice (KU steps) before the products.
constexpr int PR_MAXR = 128;

// Work-group: PGN consecutive entries of the group list (child, group of 64
// owned nodes), the groups of every child with a coarse space numbered
// consecutively, and 16 NTL right-hand sides from 64 blockIdx.y.  NTL tiles of
// 16 right-hand sides per wave (fewer when q is small; an output's arithmetic
// is the same for any NTL and PGN).  Several groups per work-group (few
// right-hand sides) spread the set-up of a work-group (box records, y staging)
// over more nodes and keep more work-groups resident in the LDS.  With active
// flags a box none of whose right-hand sides is active is skipped before any
// access.  Every branch around a barrier depends on the work-group's group
// entries only (uniform).
template <int NTL, int PGN>
__global__ void __launch_bounds__(TB) k_prolong_mfma(const BoxDev* __restrict__ child, const BoxDev* __restrict__ par,
                                                     const ParentDev* __restrict__ pd,
                                                     const int2* __restrict__ groups, int ngroups, int q,
                                                     const c128* __restrict__ C, const c128* __restrict__ y,
                                                     c128* __restrict__ u, const int* __restrict__ active) {
  extern __shared__ double2 ys[];  // ys[c][a], 16 NTL x (r + 1)
  const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
  const int c0 = blockIdx.y * 64;
  int staged = -1;
  for (int sub = 0; sub < PGN; ++sub) {
    const int gi = blockIdx.x * PGN + sub;
    if (gi >= ngroups) break;
    const int2 bg = groups[gi];
    const int box = bg.x;
    const BoxDev B = child[box];
    const int g0 = bg.y * (TB / 64) * 16;
    if (B.r == 0 || g0 >= B.n_own) continue;
    if (active) {
      bool any = false;
      for (int cc = c0; cc < q && cc < c0 + 16 * NTL; ++cc) any = any || active[B.prob * q + cc];
      if (!any) continue;
    }
    const BoxDev P = par[B.parent];
    const int rs = B.r + 1;
    if (box != staged) {
      const ParentDev D = pd[B.parent];
      __syncthreads();  // the previous box's products have read their y block
      for (int idx = threadIdx.x; idx < 16 * NTL * B.r; idx += TB) {
        const int cl = idx / B.r, a = idx - cl * B.r;
        const int c = c0 + cl;
        ys[cl * rs + a] = c < q ? y[D.yoff * q + (long long)c * D.n_c + B.cidx + a] : mk(0.0, 0.0);
      }
      __syncthreads();
      staged = box;
    }
    const int e0 = g0 + (threadIdx.x >> 6) * 16;
    if (e0 >= B.n_own) continue;
    const c128* Cb = C + B.coff;
    const int en = e0 + m;
    d4 re[NTL], im[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) re[t] = im[t] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < B.r; k0 += 4 * KU) {
      double2 cv[KU];
#pragma unroll
      for (int uu = 0; uu < KU; ++uu) {
        const int a = k0 + 4 * uu + kk;
        cv[uu] = (a < B.r && en < B.n_own) ? Cb[(long long)a * B.n_own + en] : mk(0.0, 0.0);
      }
#pragma unroll
      for (int uu = 0; uu < KU; ++uu) {
        if (k0 + 4 * uu >= B.r) break;  // steps past this box's rank skipped
        const int a = k0 + 4 * uu + kk;
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
          const double2 yv = a < B.r ? ys[(16 * t + m) * rs + a] : mk(0.0, 0.0);
          cmfma(yv, cv[uu], re[t], im[t]);
        }
      }
    }
    const int e = e0 + (lane & 15);
    if (e < B.n_own) {
      c128* ub = u + P.voff * q + owned_to_parent(B, P, e);
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
          const int c = c0 + 16 * t + 4 * sl + (lane >> 4);
          if (c < q) ub[(long long)c * P.n] = cadd(ub[(long long)c * P.n], mk(re[t][sl], im[t][sl]));
        }
    }
  }
}

// Few right-hand sides (q <= RV_MAXQ) and ranks up to 32: the restriction and
// the prolongation as vector FMA chains.  The matrix-core kernels spend 16
// right-hand-side columns of work per tile whatever q is; these do q.
// v_mfma_f64_16x16x4f64 adds its four k terms to the accumulator as a chain of
// fused multiply-adds in k order (compared bit for bit with exact rational
// arithmetic on random operands of mixed magnitude), so chains taken in the
// order of the matrix-core kernels give the same bits: a column's result does
// not depend on which of the kernels the batch width selects.
constexpr int RV_MAXQ = 4;
constexpr int RV_MAXR = 32;

// One wave per restriction chunk (RCH owned nodes): C and t staged through the
// wave's LDS slice 16 nodes at a time (coalesced loads); lane l accumulates the
// outputs (a, c) = (l & 31, (l >> 5) + 2 j).  Per output and group of four
// nodes: re += Cx tx, re += Cy ty, im += Cx ty, im += -Cy tx, each over the
// four nodes in order (the sequence of cmfma_ca in k_restrict_mfma<2>).
__global__ void __launch_bounds__(TB) k_restrict_vec(const BoxDev* __restrict__ child, const BoxDev* __restrict__ par,
                                                     const int2* __restrict__ chunks, int nitems, int q,
                                                     const c128* __restrict__ C, const c128* __restrict__ t,
                                                     c128* __restrict__ part, const int* __restrict__ active) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = blockIdx.x * (TB / 64) + wave;
  if (g >= nitems) return;
  const int2 bc = chunks[g];
  const BoxDev B = child[bc.x];
  if (active) {
    bool any = false;
    for (int cc = 0; cc < q; ++cc) any = any || active[B.prob * q + cc];
    if (!any) return;
  }
  const BoxDev P = par[B.parent];
  const int e0 = bc.y * RCH;
  const int e1 = e0 + RCH < B.n_own ? e0 + RCH : B.n_own;
  const c128* tb = t + P.voff * q;
  const c128* Cb = C + B.coff;
  __shared__ double2 cst[TB / 64][RV_MAXR * RST];
  __shared__ double2 tst[TB / 64][RV_MAXQ * RST];
  double2* cw = cst[wave];
  double2* tw = tst[wave];
  const int a = lane & 31, cl = lane >> 5;
  double re[2] = {0.0, 0.0}, im[2] = {0.0, 0.0};
  for (int k0 = e0; k0 < e1; k0 += 16) {
    const int e = k0 + (lane & 15);
    double2 cv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int aa = 4 * i + (lane >> 4);
      cv[i] = (e < e1 && aa < B.r) ? Cb[(long long)aa * B.n_own + e] : mk(0.0, 0.0);
    }
    const int ct = lane >> 4;
    const double2 tv = (e < e1 && ct < q) ? tb[(long long)ct * P.n + owned_to_parent(B, P, e)] : mk(0.0, 0.0);
    wave_lds_sync();  // the previous stage's operands have been read
#pragma unroll
    for (int i = 0; i < 8; ++i) cw[(4 * i + (lane >> 4)) * RST + (lane & 15)] = cv[i];
    tw[ct * RST + (lane & 15)] = tv;
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = cl + 2 * j;
      if (c >= q) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double2 cc[4], tt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cc[k] = cw[a * RST + 4 * u + k];
          tt[k] = tw[c * RST + 4 * u + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) re[j] = fma(cc[k].x, tt[k].x, re[j]);
#pragma unroll
        for (int k = 0; k < 4; ++k) re[j] = fma(cc[k].y, tt[k].y, re[j]);
#pragma unroll
        for (int k = 0; k < 4; ++k) im[j] = fma(cc[k].x, tt[k].y, im[j]);
#pragma unroll
        for (int k = 0; k < 4; ++k) im[j] = fma(-cc[k].y, tt[k].x, im[j]);
      }
    }
  }
  // the tile layout of k_restrict_mfma<2> with one column group: part[g][a][c], 16 columns
  c128* pb = part + (long long)g * (2 * 16) * 16;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int c = cl + 2 * j;
    if (c < q) pb[a * 16 + c] = mk(re[j], im[j]);
  }
}

// One wave per group of 64 owned nodes (lane = node), four groups per
// work-group; the box's y block staged in the wave's LDS slice.  Per output
// and group of four coarse vectors: re += yx Cx, re += -yy Cy, im += yx Cy,
// im += yy Cx, each over the four in order (the sequence of cmfma in
// k_prolong_mfma).
__global__ void __launch_bounds__(TB) k_prolong_vec(const BoxDev* __restrict__ child, const BoxDev* __restrict__ par,
                                                    const ParentDev* __restrict__ pd,
                                                    const int2* __restrict__ groups, int ngroups, int q,
                                                    const c128* __restrict__ C, const c128* __restrict__ y,
                                                    c128* __restrict__ u, const int* __restrict__ active) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gi = blockIdx.x * (TB / 64) + wave;
  if (gi >= ngroups) return;
  const int2 bg = groups[gi];
  const BoxDev B = child[bg.x];
  const int g0 = bg.y * (TB / 64) * 16;
  if (B.r == 0 || g0 >= B.n_own) return;
  if (active) {
    bool any = false;
    for (int cc = 0; cc < q; ++cc) any = any || active[B.prob * q + cc];
    if (!any) return;
  }
  const BoxDev P = par[B.parent];
  const ParentDev D = pd[B.parent];
  __shared__ double2 yst[TB / 64][RV_MAXQ * (RV_MAXR + 1)];
  double2* yw = yst[wave];
  constexpr int YR = RV_MAXR + 1;
  for (int idx = lane; idx < q * B.r; idx += 64) {
    const int c = idx / B.r, a = idx - c * B.r;
    yw[c * YR + a] = y[D.yoff * q + (long long)c * D.n_c + B.cidx + a];
  }
  wave_lds_sync();
  const int e = g0 + lane;
  const bool ve = e < B.n_own;
  const c128* Cb = C + B.coff;
  double re[RV_MAXQ], im[RV_MAXQ];
#pragma unroll
  for (int c = 0; c < RV_MAXQ; ++c) re[c] = im[c] = 0.0;
  for (int k0 = 0; k0 < B.r; k0 += 4) {
    double2 cv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      cv[k] = (k0 + k < B.r && ve) ? Cb[(long long)(k0 + k) * B.n_own + e] : mk(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < RV_MAXQ; ++c) {
      if (c >= q) break;
      double2 yv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) yv[k] = k0 + k < B.r ? yw[c * YR + k0 + k] : mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 4; ++k) re[c] = fma(yv[k].x, cv[k].x, re[c]);
#pragma unroll
      for (int k = 0; k < 4; ++k) re[c] = fma(-yv[k].y, cv[k].y, re[c]);
#pragma unroll
      for (int k = 0; k < 4; ++k) im[c] = fma(yv[k].x, cv[k].y, im[c]);
#pragma unroll
      for (int k = 0; k < 4; ++k) im[c] = fma(yv[k].y, cv[k].x, im[c]);
    }
  }
  if (ve) {
    c128* ub = u + P.voff * q + owned_to_parent(B, P, e);
#pragma unroll
    for (int c = 0; c < RV_MAXQ; ++c) {
      if (c >= q) break;
      ub[(long long)c * P.n] = cadd(ub[(long long)c * P.n], mk(re[c], im[c]));
    }
  }
}

inline int gx(long long n, int cap) {
  long long g = (n + TB - 1) / TB;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_galerkin_ac(const OpDev* ops, const BoxDev* boxes, int nbox, const BoxDev* par, const int4* dil,
                              int max_dil, int rmax, const c128* C, c128* AC, hipStream_t s) {
  if (nbox <= 0 || rmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_galerkin_ac, dim3(gx(max_dil, 256), nbox * rmax), dim3(TB), 0, s, ops, boxes, par, dil, rmax,
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

hipError_t launch_drop_negligible(const BoxDev* boxes, int nbox, int rmax, double tol, c128* C, int* drop,
                                  hipStream_t s) {
  if (nbox <= 0 || rmax <= 0) return hipSuccess;
  if (rmax > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_drop_negligible, dim3(nbox), dim3(TBD), 0, s, boxes, rmax, tol, C, drop);
  return hipGetLastError();
}

hipError_t launch_unit_dropped(const BoxDev* boxes, const ParentDev* pd, int nbox, int rmax, const int* drop,
                               c128* A, hipStream_t s) {
  if (nbox <= 0 || rmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_dropped, dim3((nbox * rmax + 255) / 256), dim3(256), 0, s, boxes, pd, nbox, rmax, drop, A);
  return hipGetLastError();
}

hipError_t launch_gj_inverse(const ParentDev* pars, int npar, int max_nc, c128* A, int* piv, c128* fcol, int* info,
                             hipStream_t s) {
  if (npar <= 0 || max_nc <= 0) return hipSuccess;
  hipError_t e = launch_fill_zero(info, (long long)sizeof(int) * npar, s);
  if (e != hipSuccess) return e;
  auto panel_shm = [](int n) {
    return sizeof(double2) * ((size_t)(GJ_NB + 1) * n + 2 * GJ_NB) + sizeof(int) * (size_t)n;
  };
  const size_t shm = panel_shm(max_nc);
  // raised once, to the largest panel (a per-call setting could be lowered by a
  // concurrent caller between another caller's setting and its launch)
  static const hipError_t raised = hipFuncSetAttribute(
      reinterpret_cast<const void*>(k_gj_panel), hipFuncAttributeMaxDynamicSharedMemorySize, (int)panel_shm(GJ_MAXN));
  if (max_nc <= GJ_MAXN && (shm <= 65536 || raised == hipSuccess)) {
    // blocked: two launches per panel of GJ_NB pivots (fcol holds the permutations)
    int* sig = reinterpret_cast<int*>(fcol);
    for (int k0 = 0; k0 < max_nc; k0 += GJ_NB) {
      hipLaunchKernelGGL(k_gj_panel, dim3(npar), dim3(1024), shm, s, pars, A, piv, sig, max_nc, k0, info);
      hipLaunchKernelGGL(k_gj_trail, dim3(max_nc, npar), dim3(256), 0, s, pars, A, sig, max_nc, k0);
    }
    hipLaunchKernelGGL(k_gj_unperm, dim3((max_nc + TB - 1) / TB, npar), dim3(TB), 0, s, pars, A, piv, max_nc);
    return hipGetLastError();
  }
  // blocks per parent: enough for one large A_c, few when there are many parents
  // (the elimination loop strides over the matrix)
  const long long nn = (long long)max_nc * max_nc;
  const int gxe = gx(nn, std::max(8, std::min(1024, 8192 / npar)));
  for (int kk = 0; kk < max_nc; ++kk) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(npar), dim3(TB), 0, s, pars, A, piv, fcol, max_nc, kk, info);
    hipLaunchKernelGGL(k_gj_elim, dim3(gxe, npar), dim3(TB), 0, s, pars, A, fcol, max_nc, kk);
  }
  hipLaunchKernelGGL(k_gj_unperm, dim3((max_nc + TB - 1) / TB, npar), dim3(TB), 0, s, pars, A, piv, max_nc);
  return hipGetLastError();
}

namespace {
// tiles of 16 coarse vectors instantiated for the restriction: 2, 4 or 8 (0: unsupported)
int restrict_tiles(int rmax) {
  const int mt = (rmax + 15) / 16;
  return mt <= 2 ? 2 : mt <= 4 ? 4 : mt <= 8 ? 8 : 0;
}
}  // namespace

int restrict_chunk_nodes() { return RCH; }

// The workspace holds, per chunk, the full padded (16 MT) x (16 ncg) tile that
// k_restrict_mfma writes.
long long restrict_workspace(int nchunks, int rmax, int q) {
  if (nchunks <= 0 || rmax <= 0 || q <= 0) return 0;
  const long long rpad = 16LL * restrict_tiles(rmax), qpad = (q + 15) / 16 * 16;
  return nchunks * rpad * qpad;
}

hipError_t launch_coarse_restrict(const BoxDev* child, int nchild, const int2* chunks, const int* cbase, int nchunks,
                                  const BoxDev* par, const ParentDev* pd, int rmax, int q, const c128* C,
                                  const c128* t, c128* part, c128* cvec, const int* active, hipStream_t s) {
  if (nchild <= 0 || nchunks <= 0 || rmax <= 0 || q <= 0) return hipSuccess;
  const int mt = restrict_tiles(rmax);
  if (mt == 0) return hipErrorInvalidValue;
  const int ncg = (q + 15) / 16;
  const long long nitems = (long long)nchunks * ncg;
  if (nitems > (1LL << 30)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nitems + TB / 64 - 1) / (TB / 64)));
  if (mt == 2 && q <= RV_MAXQ)
    hipLaunchKernelGGL(k_restrict_vec, grid, dim3(TB), 0, s, child, par, chunks, (int)nitems, q, C, t, part, active);
  else if (mt == 2)
    hipLaunchKernelGGL(k_restrict_mfma<2>, grid, dim3(TB), 0, s, child, par, chunks, (int)nitems, ncg, q, C, t, part,
                       active);
  else if (mt == 4)
    hipLaunchKernelGGL(k_restrict_mfma<4>, grid, dim3(TB), 0, s, child, par, chunks, (int)nitems, ncg, q, C, t, part,
                       active);
  else
    hipLaunchKernelGGL(k_restrict_mfma<8>, grid, dim3(TB), 0, s, child, par, chunks, (int)nitems, ncg, q, C, t, part,
                       active);
  hipLaunchKernelGGL(k_restrict_sum, dim3((rmax * q + RS_OUT - 1) / RS_OUT, nchild), dim3(RS_SEG * RS_OUT), 0, s,
                     child, pd, cbase, 16 * mt, q, ncg * 16, part, cvec);
  return hipGetLastError();
}

hipError_t launch_coarse_gemv(const ParentDev* pd, int npar, int max_nc, int q, const c128* Ainv,
                              const c128* cvec, c128* y, hipStream_t s) {
  if (npar <= 0 || max_nc <= 0 || q <= 0) return hipSuccess;
  const int mtiles = (max_nc + 15) / 16, ntiles = (q + 15) / 16;
  hipLaunchKernelGGL(k_coarse_gemm, dim3(mtiles * ntiles, npar), dim3(TB), 0, s, pd, q, ntiles, Ainv, cvec, y);
  return hipGetLastError();
}

int prolong_group_nodes() { return (TB / 64) * 16; }

hipError_t launch_coarse_prolong(const BoxDev* child, const int2* groups, int ngroups, int rmax, const BoxDev* par,
                                 const ParentDev* pd, int q, const c128* C, const c128* y, c128* u,
                                 const int* active, hipStream_t s) {
  if (ngroups <= 0 || q <= 0) return hipSuccess;
  if (rmax > PR_MAXR) return hipErrorInvalidValue;
  if (q <= RV_MAXQ && rmax <= RV_MAXR) {
    hipLaunchKernelGGL(k_prolong_vec, dim3((ngroups + TB / 64 - 1) / (TB / 64)), dim3(TB), 0, s, child, par, pd, groups,
                       ngroups, q, C, y, u, active);
    return hipGetLastError();
  }
  const int ntl = q <= 16 ? 1 : q <= 32 ? 2 : 4;
  const size_t shm = sizeof(double2) * 16 * ntl * (size_t)(rmax + 1);
  // raised once, to the largest rank (see launch_gj_inverse)
  static const hipError_t raised = [] {
    const int most = (int)(sizeof(double2) * 64 * (PR_MAXR + 1));
    for (const void* k : {reinterpret_cast<const void*>(k_prolong_mfma<1, 4>),
                          reinterpret_cast<const void*>(k_prolong_mfma<2, 4>),
                          reinterpret_cast<const void*>(k_prolong_mfma<4, 1>)}) {
      const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, most);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }();
  if (shm > 65536 && raised != hipSuccess) return raised;
  // few right-hand sides: four node groups per work-group; 64: one (enough work-groups to fill the chip)
  const int pgn = ntl == 4 ? 1 : 4;
  const dim3 grid((ngroups + pgn - 1) / pgn, (q + 63) / 64);
  if (ntl == 1)
    hipLaunchKernelGGL((k_prolong_mfma<1, 4>), grid, dim3(TB), shm, s, child, par, pd, groups, ngroups, q, C, y, u,
                       active);
  else if (ntl == 2)
    hipLaunchKernelGGL((k_prolong_mfma<2, 4>), grid, dim3(TB), shm, s, child, par, pd, groups, ngroups, q, C, y, u,
                       active);
  else
    hipLaunchKernelGGL((k_prolong_mfma<4, 1>), grid, dim3(TB), shm, s, child, par, pd, groups, ngroups, q, C, y, u,
                       active);
  return hipGetLastError();
}
