// Leaf subdomain solves A~_i x = b (the local impedance problems of eq. (sub1))
// with the two-ended ("twisted") block factorisation of k_leaf.hip.
//
// Box matrix in line-major order (line j = the ny nodes with p = p0 + j):
// block tridiagonal, diagonal blocks tridiagonal, line-to-line couplings
// diagonal.  With m = nx / 2 the factor keeps one dense b x b inverse per line
// (b = ny):
//   top     G_j = S_j^{-1},  S_0 = A_00,  S_j = A_jj - A_{j,j-1} S_{j-1}^{-1} A_{j-1,j}   (j < m)
//   bottom  G_j = T_j^{-1},  T_{nx-1} = A,  T_j = A_jj - A_{j,j+1} T_{j+1}^{-1} A_{j+1,j}   (j > m)
//   middle  G_m = (A_mm - A_{m,m-1} S_{m-1}^{-1} A_{m-1,m} - A_{m,m+1} T_{m+1}^{-1} A_{m+1,m})^{-1}.
// A solve is two launches.  Phase 1 runs both halves towards the middle,
//   w_j = G_j (b_j - A_{j,j-1} w_{j-1})   (j = 0 .. m-1)
//   v_j = G_j (b_j - A_{j,j+1} v_{j+1})   (j = nx-1 .. m+1),
// phase 2 solves the middle line and substitutes outwards,
//   x_m = G_m (b_m - A_{m,m-1} w_{m-1} - A_{m,m+1} v_{m+1})
//   x_j = w_j - G_j A_{j,j+1} x_{j+1}  (j < m),   x_j = v_j - G_j A_{j,j-1} x_{j-1}  (j > m).
// The sequential chain is nx + 1 dense steps instead of 2 nx - 1, and every
// (leaf, half) pair is an independent work unit.
//
// One work-group = one (leaf, half) unit and QB right-hand sides; NW waves.
// Thread tile: TM rows x R columns of G_j x QB right-hand sides.  Lane bits
// {0, 4, 5} select one of KS = 8 column slices (k = ks R + r), lane bits
// {1, 2, 3} and the wave select the row group (rows i = rg + 8 NW t).  The
// slice partial sums meet through cross-lane swaps inside the wave (gfx950
// permlane32/permlane16 swaps, DPP quad permute), halving the values held per
// lane at each stage, so no partial sums pass through LDS; the right-hand
// side tile y_j lives in LDS (double-buffered, one barrier per line) and the
// next line's G_j slice is loaded into registers while the current one is
// applied.  The summation order of every output depends on b (through R)
// only, so a right-hand side gives the same bits in any batch.
#include "kernels.h"

namespace {

constexpr int KS = 8;

// ---- cross-lane sums.  sum_x32(a, b): lanes 0..31 get a(l) + a(l + 32),
// lanes 32..63 get b(l - 32) + b(l).  sum_x16 likewise across the 16-lane
// halves of each 32-lane half.  sum_x1 halves across lane pairs (l, l ^ 1):
// even lanes get a(l) + a(l + 1), odd lanes b(l - 1) + b(l).
__device__ __forceinline__ float sum_x32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double sum_x32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float sum_x16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double sum_x16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
// DPP quad permute [1, 0, 3, 2]: the value of lane l ^ 1
__device__ __forceinline__ float xor1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, false));
}
__device__ __forceinline__ double xor1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0xb1, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0xb1, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <typename S>
__device__ __forceinline__ S sum_x1(S a, S b, bool odd) {
  const S keep = odd ? b : a, send = odd ? a : b;
  return keep + xor1(send);
}

// Reduction of v[M0] over the KS = 8 slices of a row group: stages over lane
// bits 5, 4, 0.  A stage with an even count halves it (the lane keeps the half
// its bit selects); an odd count is summed on both lanes.
template <int M>
struct Halve {
  static constexpr int next = (M % 2 == 0) ? M / 2 : M;
  static constexpr bool odd = (M % 2) != 0;
};

template <typename CT, int M0>
__device__ __forceinline__ void reduce_slices(CT (&v)[M0], int lane) {
  constexpr int M1 = Halve<M0>::next, M2 = Halve<M1>::next, M3 = Halve<M2>::next;
  // bit 5
  if constexpr (Halve<M0>::odd) {
#pragma unroll
    for (int t = 0; t < M0; ++t) v[t] = mk(sum_x32(v[t].x, v[t].x), sum_x32(v[t].y, v[t].y));
  } else {
#pragma unroll
    for (int t = 0; t < M1; ++t) v[t] = mk(sum_x32(v[t].x, v[t + M1].x), sum_x32(v[t].y, v[t + M1].y));
  }
  // bit 4
  if constexpr (Halve<M1>::odd) {
#pragma unroll
    for (int t = 0; t < M1; ++t) v[t] = mk(sum_x16(v[t].x, v[t].x), sum_x16(v[t].y, v[t].y));
  } else {
#pragma unroll
    for (int t = 0; t < M2; ++t) v[t] = mk(sum_x16(v[t].x, v[t + M2].x), sum_x16(v[t].y, v[t + M2].y));
  }
  // bit 0
  const bool odd = lane & 1;
  if constexpr (Halve<M2>::odd) {
#pragma unroll
    for (int t = 0; t < M2; ++t) v[t] = mk(v[t].x + xor1(v[t].x), v[t].y + xor1(v[t].y));
  } else {
#pragma unroll
    for (int t = 0; t < M3; ++t)
      v[t] = mk(sum_x1(v[t].x, v[t + M3].x, odd), sum_x1(v[t].y, v[t + M3].y, odd));
  }
}

// Which reduced values a lane holds: flat indices base + t (t < M3) of the
// TM x QB tile; lanes that hold the same set after odd stages split the
// epilogue work by t % dups == dup.
template <int M0>
struct SlotMap {
  static constexpr int M1 = Halve<M0>::next, M2 = Halve<M1>::next, M3 = Halve<M2>::next;
  static constexpr int dups = (Halve<M0>::odd ? 2 : 1) * (Halve<M1>::odd ? 2 : 1) * (Halve<M2>::odd ? 2 : 1);
  __device__ static void lane_info(int lane, int& base, int& dup) {
    const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b0 = lane & 1;
    base = 0;
    dup = 0;
    int mult = 1;
    if (Halve<M0>::odd) { dup += b5 * mult; mult *= 2; } else base += b5 * M1;
    if (Halve<M1>::odd) { dup += b4 * mult; mult *= 2; } else base += b4 * M2;
    if (Halve<M2>::odd) { dup += b0 * mult; } else base += b0 * M3;
  }
};

// PHASE 1: outer lines towards the middle; PHASE 2: middle line and
// back-substitution (a template argument, so profiles list the phases apart)
template <typename T, int QB, int TM, int R, int NW, bool PF, int PHASE>
__global__ void __launch_bounds__(64 * NW)
    k_sweep(const OpDev* __restrict__ ops, const BoxDev* __restrict__ leaves, const int* __restrict__ lidx,
            int nunit, int nchunk, int q,
            const typename cvec<T>::type* __restrict__ G, const c128* __restrict__ rhs, c128* __restrict__ x,
            c128* __restrict__ edge, int edge_ld, const BoxDev* __restrict__ par, c128* __restrict__ out,
            const int* __restrict__ active) {
  typedef typename cvec<T>::type CT;
  constexpr int phase = PHASE;
  constexpr int NT = 64 * NW, RG = 8 * NW, M0 = TM * QB;
  constexpr int YS = R * QB + 1;  // LDS stride of a column slice (odd: slices start on different banks)
  typedef SlotMap<M0> SM;
  constexpr int MF = SM::M3;
  __shared__ CT ybuf[2][KS * YS];

  int unit, chunk;
  if ((nunit & 7) == 0) {
    // dispatch is round-robin over the 8 XCDs: keep all chunks of a unit on one XCD (shared L2 copy of G)
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    unit = xcd + 8 * (slot / nchunk);
    chunk = slot % nchunk;
  } else {
    unit = blockIdx.x / nchunk;
    chunk = blockIdx.x % nchunk;
  }
  const int leaf = lidx[unit >> 1], half = unit & 1;
  const BoxDev B = leaves[leaf];
  const OpDev op = ops[B.prob];
  const int b = B.ny, nx = B.nx, m = nx >> 1;
  const int n_top = m, n_bot = nx - 1 - m;
  // lines of this unit in this phase: line(s) = l0 + dl * s, s < ns
  int ns, l0, dl;
  if (phase == 1) {
    ns = half ? n_bot : n_top;
    l0 = half ? nx - 1 : 0;
    dl = half ? -1 : 1;
  } else {
    ns = half ? (n_bot > 0 ? n_bot + 1 : 0) : n_top + 1;
    l0 = m;
    dl = half ? 1 : -1;
  }
  if (ns == 0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ks = (lane & 1) | (((lane >> 4) & 1) << 1) | (((lane >> 5) & 1) << 2);
  const int rgi = wave * 8 + ((lane >> 1) & 7);
  const int c0 = chunk * QB;
  if (active) {
    // right-hand sides of this problem that still iterate (the others' outputs are not used)
    bool any = false;
    for (int c = 0; c < QB && c0 + c < q; ++c) any = any || active[B.prob * q + c0 + c];
    if (!any) return;
  }
  const long long base = B.voff * q;
  // right-hand side: the box's own vector, or (par given) read in place from
  // the parent's vector; node (line, i) of column c at rbase + c rcol + line rrow + i
  long long rbase = base, rcol = B.n;
  int rrow = b;
  if (par) {
    const BoxDev P = par[B.parent];
    rbase = P.voff * q + (long long)(B.p0 - P.p0) * P.ny + (B.q0 - P.q0);
    rcol = P.n;
    rrow = P.ny;
  }
  const long long bb = (long long)b * b;
  const CT* Gl = G + B.goff;
  const CT zero = mk((T)0, (T)0);

  // reduced outputs held by this lane
  int sbase, sdup;
  SM::lane_info(lane, sbase, sdup);
  int orow[MF], ocol[MF];
  bool own[MF];
#pragma unroll
  for (int t = 0; t < MF; ++t) {
    const int f = sbase + t;
    const int tm = f / QB, c = f % QB;
    orow[t] = rgi + RG * tm;
    ocol[t] = c;
    own[t] = (t % SM::dups) == sdup && orow[t] < b && c0 + c < q;
  }
  // clamped addresses for branch-free prefetches (used only where own[t])
  long long oaddr[MF], raddr[MF];
#pragma unroll
  for (int t = 0; t < MF; ++t) {
    const int i = orow[t] < b ? orow[t] : b - 1;
    const int c = c0 + ocol[t] < q ? c0 + ocol[t] : q - 1;
    oaddr[t] = base + (long long)c * B.n + i;
    raddr[t] = rbase + (long long)c * rcol + i;
  }

  // G slice of the first line into registers (PF: the next line's slice is
  // loaded while the current one is applied; else each entry is loaded at use)
  CT g[PF ? TM * R : 1];
  if constexpr (PF) {
    const CT* Gj = Gl + (long long)l0 * bb;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = ks * R + r;
        g[tm * R + r] = Gj[(long long)k * b + rgi + RG * tm];
      }
  }
  for (int e = tid; e < 2 * KS * YS; e += NT) (&ybuf[0][0])[e] = zero;
  lds_barrier();
  // y of the first step
  for (int e = tid; e < b * QB; e += NT) {
    const int i = e % b, c = e / b;
    double2 v = mk(0.0, 0.0);
    if (c0 + c < q) {
      v = rhs[rbase + (long long)(c0 + c) * rcol + (long long)l0 * rrow + i];
      if (phase == 2) {
        const int p = B.p0 + m, qq = B.q0 + i;
        if (n_top > 0) {
          const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, -1, 0);
          v = csub(v, cmul(a, edge[((long long)(leaf * 2) * q + c0 + c) * edge_ld + i]));
        }
        if (n_bot > 0) {
          const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, 1, 0);
          v = csub(v, cmul(a, edge[((long long)(leaf * 2 + 1) * q + c0 + c) * edge_ld + i]));
        }
      }
    }
    ybuf[0][(i / R) * YS + (i % R) * QB + c] = from_c128<T>(v);
  }
  lds_barrier();

  for (int s = 0; s < ns; ++s) {
    const int j = l0 + dl * s;
    const bool more = s + 1 < ns;
    const int jn = more ? j + dl : j;
    // epilogue operands: phase 1 needs b_{j+dl}; phase 2 (s > 0) needs w_j / v_j
    double2 pre[MF];
    if (phase == 1) {
#pragma unroll
      for (int t = 0; t < MF; ++t) pre[t] = rhs[raddr[t] + (long long)jn * rrow];
    } else {
#pragma unroll
      for (int t = 0; t < MF; ++t) pre[t] = x[oaddr[t] + (long long)j * b];
    }
    // issued here, consumed in the epilogue: kept ahead of the next line's G
    // loads so that waiting for them leaves those in flight
    __builtin_amdgcn_sched_barrier(0);
    // y rows k >= b are zero in LDS, so the G entries read past a line's b
    // columns (finite: the next columns, or the zeroed tail) add nothing
    const CT* Gn = Gl + (long long)jn * bb;
    const CT* Gc = Gl + (long long)j * bb;
    const CT* ys = &ybuf[s & 1][ks * YS];
    CT acc[M0];
#pragma unroll
    for (int t = 0; t < M0; ++t) acc[t] = zero;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      CT yv[QB];
#pragma unroll
      for (int c = 0; c < QB; ++c) yv[c] = ys[r * QB + c];
      const int k = ks * R + r;
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        if constexpr (PF) {
#pragma unroll
          for (int c = 0; c < QB; ++c) acc[tm * QB + c] = cfma(g[tm * R + r], yv[c], acc[tm * QB + c]);
          g[tm * R + r] = Gn[(long long)k * b + rgi + RG * tm];
        } else {
          const CT v = Gc[(long long)k * b + rgi + RG * tm];
          const CT gv = k < b ? v : zero;
#pragma unroll
          for (int c = 0; c < QB; ++c) acc[tm * QB + c] = cfma(gv, yv[c], acc[tm * QB + c]);
        }
      }
    }
    reduce_slices<CT, M0>(acc, lane);
    CT* yn = &ybuf[(s + 1) & 1][0];
#pragma unroll
    for (int t = 0; t < MF; ++t) {
      if (!own[t]) continue;
      const int i = orow[t], c = ocol[t];
      const double2 r = to_c128(acc[t]);
      double2 xv;
      if (phase == 1 || s == 0) {
        xv = r;  // w_j, v_j or x_m
      } else {
        xv = csub(pre[t], r);  // x_j = w_j - G_j A x_{j -+ 1}
      }
      const long long at = oaddr[t] + (long long)j * b;
      if (phase == 1) {
        x[at] = xv;
        if (!more) edge[((long long)(2 * leaf + half) * q + c0 + c) * edge_ld + i] = xv;
      } else if (s > 0 || half == 0) {
        if (!out) {
          x[at] = xv;
        } else {
          // the restricted prolongation: owned nodes straight into the parent's vector
          const int p = B.p0 + j, qq = B.q0 + i;
          if (p >= B.op0 && p <= B.op1 && qq >= B.oq0 && qq <= B.oq1) out[raddr[t] + (long long)j * rrow] = xv;
        }
      }
      if (more) {
        const double2 a = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, B.p0 + jn, B.q0 + i, j - jn, 0);
        const double2 yv = phase == 1 ? csub(pre[t], cmul(a, xv)) : cmul(a, xv);
        yn[(i / R) * YS + (i % R) * QB + c] = from_c128<T>(yv);
      }
    }
    lds_barrier();
  }
}

template <typename T, int QB, int TM, int R, int NW, bool PF>
hipError_t launch_sweep(const OpDev* ops, const BoxDev* leaves, const int* lidx, int count, int q,
                        const typename cvec<T>::type* G, const c128* rhs, c128* x, c128* edge, int edge_ld,
                        const BoxDev* par, c128* out, const int* active, hipStream_t s) {
  const int nchunk = (q + QB - 1) / QB, nunit = 2 * count;
  const dim3 grid(nunit * nchunk), block(64 * NW);
  hipLaunchKernelGGL((k_sweep<T, QB, TM, R, NW, PF, 1>), grid, block, 0, s, ops, leaves, lidx, nunit, nchunk, q, G,
                     rhs, x, edge, edge_ld, par, out, active);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sweep<T, QB, TM, R, NW, PF, 2>), grid, block, 0, s, ops, leaves, lidx, nunit, nchunk, q, G,
                     rhs, x, edge, edge_ld, par, out, active);
  return hipGetLastError();
}

// Column count QB per work-group: given (1, 2, 4), else enough work-groups to
// cover the chip and up to four columns per group to amortise the G_j stream.
// QB does not change any column's arithmetic.
template <typename T, int TM, int R, int NW, bool PF>
hipError_t launch_qb(const OpDev* ops, const BoxDev* leaves, const int* lidx, int count, int q, int qb,
                     const typename cvec<T>::type* G, const c128* rhs, c128* x, c128* edge, int edge_ld,
                     const BoxDev* par, c128* out, const int* active, hipStream_t s) {
  const long long units = 2LL * count;
  if (qb <= 0) qb = (q >= 4 && units * ((q + 3) / 4) >= 256) ? 4 : (q >= 2 && units * ((q + 1) / 2) >= 128) ? 2 : 1;
  if (qb == 4)
    return launch_sweep<T, 4, TM, R, NW, PF>(ops, leaves, lidx, count, q, G, rhs, x, edge, edge_ld, par, out, active, s);
  if (qb == 2)
    return launch_sweep<T, 2, TM, R, NW, PF>(ops, leaves, lidx, count, q, G, rhs, x, edge, edge_ld, par, out, active, s);
  return launch_sweep<T, 1, TM, R, NW, PF>(ops, leaves, lidx, count, q, G, rhs, x, edge, edge_ld, par, out, active, s);
}

}  // namespace

// Shape buckets by leaf width b: R = ceil(b / 8) rounded up to the bucket,
// rows covered by 8 NW row groups of TM rows.  A leaf's bucket depends on its
// own width only, so a column's arithmetic is the same in any batch and for
// any q.
int leaf_sweep_bucket(int ny) {
  if (ny <= 8) return 0;
  if (ny <= 16) return 1;
  if (ny <= 40) return 2;
  if (ny <= 72) return 3;
  if (ny <= 144) return 4;
  if (ny <= 256) return 5;
  return -1;
}

template <typename T>
hipError_t launch_leaf_solve(const OpDev* ops, const BoxDev* leaves, const int* lidx, int count, int bucket,
                             int edge_ld, int q, int qb, const typename cvec<T>::type* G, const c128* rhs, c128* x,
                             c128* edge, const BoxDev* par, c128* out, const int* active, hipStream_t s) {
  if (count <= 0 || q <= 0) return hipSuccess;
  switch (bucket) {
    case 0: return launch_qb<T, 1, 1, 1, true>(ops, leaves, lidx, count, q, qb, G, rhs, x, edge, edge_ld, par, out, active, s);
    case 1: return launch_qb<T, 2, 2, 1, true>(ops, leaves, lidx, count, q, qb, G, rhs, x, edge, edge_ld, par, out, active, s);
    case 2: return launch_qb<T, 5, 5, 1, true>(ops, leaves, lidx, count, q, qb, G, rhs, x, edge, edge_ld, par, out, active, s);
    case 3: return launch_qb<T, 3, 9, 3, true>(ops, leaves, lidx, count, q, qb, G, rhs, x, edge, edge_ld, par, out, active, s);
    case 4:
      // the 3 x 18 G slice stays in registers in complex64 only
      return launch_qb<T, 3, 18, 6, sizeof(T) == 4>(ops, leaves, lidx, count, q, qb, G, rhs, x, edge, edge_ld, par,
                                                    out, active, s);
    case 5:  // loads G at use
      return launch_qb<T, 4, 32, 8, false>(ops, leaves, lidx, count, q, qb, G, rhs, x, edge, edge_ld, par, out, active, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_leaf_solve<double>(const OpDev*, const BoxDev*, const int*, int, int, int, int, int,
                                              const c128*, const c128*, c128*, c128*, const BoxDev*, c128*,
                                              const int*, hipStream_t);
template hipError_t launch_leaf_solve<float>(const OpDev*, const BoxDev*, const int*, int, int, int, int, int,
                                             const c64*, const c128*, c128*, c128*, const BoxDev*, c128*,
                                             const int*, hipStream_t);
