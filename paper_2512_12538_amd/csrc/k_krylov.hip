// Device side of the outer loops: batched inner products with a fixed
// reduction tree (the split into blocks depends on the vector length only, so
// a right-hand side gets bit-identical results alone and inside any batch),
// the Gram-Schmidt updates, and the per-right-hand-side GMRES bookkeeping
// (Givens rotations of the Hessenberg column, the convergence test, the small
// triangular solve).  The convergence decision is taken on the device so the
// host can poll it without draining the stream.
#include "kernels.h"

namespace {

constexpr int TB = 256;
constexpr int CHUNK = 1024;  // nodes per partial sum
constexpr int MAXNB = 512;
constexpr int KG = 8;        // inner products per block

inline int nblocks(long long n) {
  long long nb = (n + CHUNK - 1) / CHUNK;
  if (nb < 1) nb = 1;
  if (nb > MAXNB) nb = MAXNB;
  return (int)nb;
}

constexpr int EPT = CHUNK / TB;  // elements per thread and pass over a block's chunk
constexpr int NXCD = 8;          // XCDs; hardware block i runs on XCD i mod 8

// Krylov basis loads: the basis of a batch is far larger than the caches and
// each vector is read once per pass, so these loads bypass them.
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldnt(const c128* p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return mk(v.x, v.y);
}

// ---- wave reductions without LDS: gfx950 permlane32/permlane16 swaps for
// lane bits 5 and 4, DPP for bits 0..3.
__device__ __forceinline__ double dpp_d(double v, int ctrl_sel) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  switch (ctrl_sel) {
    case 0:  // quad_perm [1, 0, 3, 2]: lane ^ 1
      lo = __builtin_amdgcn_update_dpp(0, lo, 0xb1, 0xf, 0xf, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0xb1, 0xf, 0xf, false);
      break;
    case 1:  // quad_perm [2, 3, 0, 1]: lane ^ 2
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x4e, 0xf, 0xf, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x4e, 0xf, 0xf, false);
      break;
    case 2:  // row_ror:4
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x124, 0xf, 0xf, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x124, 0xf, 0xf, false);
      break;
    default:  // row_ror:8
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x128, 0xf, 0xf, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x128, 0xf, 0xf, false);
      break;
  }
  return __hiloint2double(hi, lo);
}
// lanes < 32: a(l) + a(l + 32); lanes >= 32: b(l - 32) + b(l)  (likewise across 16-lane halves)
__device__ __forceinline__ double swapsum32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double swapsum16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
// sum over the lanes that share bits 4 and 5 (bits 0..3 summed)
// (halve0: even lanes keep v, odd lanes keep other, each summed with its partner's)
__device__ __forceinline__ double sum16(double v, bool halve0, double other) {
  if (halve0) {
    const bool odd = threadIdx.x & 1;
    const double keep = odd ? other : v, send = odd ? v : other;
    v = keep + dpp_d(send, 0);
  } else {
    v += dpp_d(v, 0);
  }
  v += dpp_d(v, 1);
  v += dpp_d(v, 2);
  v += dpp_d(v, 3);
  return v;
}

// Block sums of KG = 8 complex values per thread, in a fixed tree.  Lane bits
// 5, 4 and 0 halve the eight values (lane keeps the half its bit selects), bits
// 1..3 are summed by DPP; the four waves meet in LDS.  Thread t < 8 returns
// the block sum of value t.
__device__ __forceinline__ double2 block_sum8(double2 (&a)[KG], double2* red) {
  double2 v4[4], v2[2];
#pragma unroll
  for (int t = 0; t < 4; ++t) v4[t] = mk(swapsum32(a[t].x, a[t + 4].x), swapsum32(a[t].y, a[t + 4].y));
#pragma unroll
  for (int t = 0; t < 2; ++t) v2[t] = mk(swapsum16(v4[t].x, v4[t + 2].x), swapsum16(v4[t].y, v4[t + 2].y));
  const double2 v = mk(sum16(v2[0].x, true, v2[1].x), sum16(v2[0].y, true, v2[1].y));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + (lane & 1);
  if ((lane & 0xe) == 0) red[wave * KG + t] = v;
  __syncthreads();
  double2 r = mk(0.0, 0.0);
  if (threadIdx.x < KG) {
#pragma unroll
    for (int w = 0; w < TB / 64; ++w) r = cadd(r, red[w * KG + threadIdx.x]);
  }
  __syncthreads();
  return r;
}

// Block sum of one real value per thread; thread 0 returns it.
__device__ __forceinline__ double block_sum1(double v, double* red) {
  v = swapsum32(v, v);
  v = swapsum16(v, v);
  v = sum16(v, false, 0.0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < TB / 64; ++w) r += red[w];
  }
  __syncthreads();
  return r;
}

// Chunk g of the outer-loop systems: system b, its elements [lo, hi) relative
// to the segment start (nb[b] chunks of equal length per system, the last one
// shorter), so the split depends on the system's length only.
struct Chunk {
  int b, blk;
  long long off, lo, hi;
};
__device__ __forceinline__ Chunk chunk_of(const SegDev& sg, int g) {
  const int2 cb = sg.chunk[g];
  Chunk c;
  c.b = cb.x;
  c.blk = cb.y;
  const long long len = sg.len[c.b];
  const int nbk = sg.nb[c.b];
  const long long per = (len + nbk - 1) / nbk;
  c.off = sg.off[c.b];
  c.lo = c.blk * per;
  c.hi = c.lo + per < len ? c.lo + per : len;
  return c;
}

// partial[blk*S1 + k*S + b] = sum over chunk blk of system b of conj(V_k[b]) W[b],
// KG consecutive k per block so that W is read once per KG products; each
// thread keeps KG x EPT basis loads in flight.  With wnorm, the first group
// also accumulates |W[b]|^2 into row nk.  Systems with skip[b] == 0 are left
// untouched (skip may be null).  S1 = (nk + wnorm) * S: the final sums read
// consecutive entries per chunk index.  One-dimensional XCD-aware grid:
// logical block (g * NKG + kg), contiguous per XCD, so the groups that share a
// chunk of W run on one XCD and read it from its L2.
__global__ void __launch_bounds__(TB) k_dot_partial(int nk, SegDev sg, int S1, const c128* __restrict__ V,
                                                    long long vstride, const c128* __restrict__ W,
                                                    c128* __restrict__ partial, int wnorm,
                                                    const int* __restrict__ skip) {
  const int nkg = (nk + KG - 1) / KG;
  const int lb = (blockIdx.x % NXCD) * (gridDim.x / NXCD) + blockIdx.x / NXCD;
  if (lb >= sg.G * nkg) return;
  const int kg = lb % nkg;
  const Chunk ch = chunk_of(sg, lb / nkg);
  const int b = ch.b, blk = ch.blk, k0 = kg * KG;
  if (skip && !skip[b]) return;
  const long long lo = ch.lo, hi = ch.hi;
  const c128* w = W + ch.off;
  const c128* vb = V + ch.off;
  const bool wn = wnorm && k0 == 0;
  const int kn = nk - k0 < KG ? nk - k0 : KG;
  double2 acc[KG];
  double nw = 0.0;
#pragma unroll
  for (int t = 0; t < KG; ++t) acc[t] = mk(0.0, 0.0);
  for (long long i0 = lo; i0 < hi; i0 += CHUNK) {
    double2 wv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const long long i = i0 + threadIdx.x + (long long)e * TB;
      wv[e] = i < hi ? w[i] : mk(0.0, 0.0);
    }
    double2 vv[KG][EPT];
#pragma unroll
    for (int t = 0; t < KG; ++t)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const long long i = i0 + threadIdx.x + (long long)e * TB;
        vv[t][e] = (t < kn && i < hi) ? ldnt(vb + (k0 + t) * vstride + i) : mk(0.0, 0.0);
      }
#pragma unroll
    for (int t = 0; t < KG; ++t)
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[t] = cfmac(vv[t][e], wv[e], acc[t]);
    if (wn) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) nw += cabs2(wv[e]);
    }
  }
  __shared__ double2 red[(TB / 64) * KG];
  const double2 r = block_sum8(acc, red);
  const int S = sg.S;
  if (threadIdx.x < kn) partial[(long long)blk * S1 + (k0 + threadIdx.x) * S + b] = r;
  if (wn) {
    const double rn = block_sum1(nw, reinterpret_cast<double*>(red));
    if (threadIdx.x == 0) partial[(long long)blk * S1 + nk * S + b] = mk(rn, 0.0);
  }
}

// out[t] = sum over the chunks of system t % S of partial[blk*nkq + t].
// Work-group: 64 outputs (lanes) x DF_SEG waves; wave k sums the chunks k,
// k + DF_SEG, ... in turn, then wave 0 adds the DF_SEG partial sums in wave
// order.  The order depends on the system's chunk count only.
constexpr int DF_SEG = 16;
__global__ void __launch_bounds__(64 * DF_SEG) k_dot_final(int nkq, int S, const int* __restrict__ nb,
                                                           const c128* __restrict__ partial, c128* __restrict__ out,
                                                           const int* __restrict__ skip) {
  const int lane = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const bool live = t < nkq && (!skip || skip[t % S]);
  double2 acc = mk(0.0, 0.0);
  if (live) {
    const int NB = nb[t % S];
    int blk = sg;
    for (; blk + 3 * DF_SEG < NB; blk += 4 * DF_SEG) {
      const double2 v0 = partial[(long long)blk * nkq + t], v1 = partial[(long long)(blk + DF_SEG) * nkq + t],
                    v2 = partial[(long long)(blk + 2 * DF_SEG) * nkq + t],
                    v3 = partial[(long long)(blk + 3 * DF_SEG) * nkq + t];
      acc = cadd(cadd(cadd(cadd(acc, v0), v1), v2), v3);
    }
    for (; blk < NB; blk += DF_SEG) acc = cadd(acc, partial[(long long)blk * nkq + t]);
  }
  __shared__ double2 red[DF_SEG][64];
  red[sg][lane] = acc;
  __syncthreads();
  if (sg == 0 && live) {
    double2 r = red[0][lane];
#pragma unroll
    for (int k = 1; k < DF_SEG; ++k) r = cadd(r, red[k][lane]);
    out[t] = r;
  }
}

// W[b] -= sum_k V_k[b] h[k*S + b] over one chunk per work-group; optionally the
// chunk sums of |W[b]|^2 after the update (npart[blk*S + b]).  The
// coefficients are uniform per work-group (scalar loads); eight basis vectors
// x EPT elements are loaded per thread before they are applied.
__global__ void __launch_bounds__(TB) k_basis_update(int nk, SegDev sg, const c128* __restrict__ V,
                                                     long long vstride, const c128* __restrict__ h,
                                                     c128* __restrict__ W, c128* __restrict__ npart,
                                                     const int* __restrict__ skip) {
  const Chunk ch = chunk_of(sg, blockIdx.x);
  const int b = ch.b, blk = ch.blk, S = sg.S;
  if (skip && !skip[b]) return;
  const long long lo = ch.lo, hi = ch.hi;
  const c128* vb = V + ch.off;
  c128* wb = W + ch.off;
  double nrm = 0.0;
  for (long long i0 = lo; i0 < hi; i0 += CHUNK) {
    double2 w[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const long long i = i0 + threadIdx.x + (long long)e * TB;
      w[e] = i < hi ? wb[i] : mk(0.0, 0.0);
    }
    int k = 0;
    for (; k + KG <= nk; k += KG) {
      double2 vv[KG][EPT];
#pragma unroll
      for (int t = 0; t < KG; ++t)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const long long i = i0 + threadIdx.x + (long long)e * TB;
          vv[t][e] = i < hi ? ldnt(vb + (k + t) * vstride + i) : mk(0.0, 0.0);
        }
#pragma unroll
      for (int t = 0; t < KG; ++t) {
        const double2 hk = h[(k + t) * S + b];
#pragma unroll
        for (int e = 0; e < EPT; ++e) w[e] = csub(w[e], cmul(vv[t][e], hk));
      }
    }
    for (; k < nk; ++k) {
      const double2 hk = h[k * S + b];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const long long i = i0 + threadIdx.x + (long long)e * TB;
        const double2 v = i < hi ? ldnt(vb + k * vstride + i) : mk(0.0, 0.0);
        w[e] = csub(w[e], cmul(v, hk));
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const long long i = i0 + threadIdx.x + (long long)e * TB;
      if (i < hi) {
        wb[i] = w[e];
        nrm += cabs2(w[e]);
      }
    }
  }
  if (npart) {
    __shared__ double red[TB / 64];
    const double r = block_sum1(nrm, red);
    if (threadIdx.x == 0) npart[(long long)blk * S + b] = mk(r, 0.0);
  }
}

// Second Gram-Schmidt pass wanted when the first one cancelled more than a
// factor eta: |w'|^2 < eta^2 |w|^2 (w0n2 = |w|^2 before, w1n2 = |w'|^2 after).
// Columns that skip it get h2 = 0 so that h1 + h2 stays the projection.
__global__ void k_reorth_flag(int q, int nk, const c128* __restrict__ w0n2, const c128* __restrict__ w1n2, double eta2,
                              int* __restrict__ need, c128* __restrict__ h2, const int* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= q) return;
  const int nd = (!active || active[b]) && (eta2 >= 1.0 || w1n2[b].x < eta2 * w0n2[b].x);
  need[b] = nd;
  if (!nd)
    for (int k = 0; k < nk; ++k) h2[k * q + b] = mk(0.0, 0.0);
}

__global__ void __launch_bounds__(TB) k_normalize(SegDev sg, const c128* __restrict__ nrm2,
                                                  const c128* __restrict__ x, c128* __restrict__ y,
                                                  double* __restrict__ nrm, const int* __restrict__ skip) {
  const Chunk ch = chunk_of(sg, blockIdx.x);
  if (skip && !skip[ch.b]) return;
  const double nv = sqrt(fmax(nrm2[ch.b].x, 0.0));
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  if (ch.blk == 0 && threadIdx.x == 0 && nrm) nrm[ch.b] = nv;
  for (long long i = ch.lo + threadIdx.x; i < ch.hi; i += TB) y[ch.off + i] = cscale(x[ch.off + i], inv);
}

// One Arnoldi column per right-hand side: H[:, j] = h1 + h2, H[j+1, j] = ||w||,
// previous rotations, a new rotation zeroing H[j+1, j], the update of g, and
// the stopping test |g_{j+1}| < thr[b] or iters[b] >= maxit.
// Layout per rhs b: H[b][(m+1)*col + row], cs/sn[b][m], g[b][m+1].
// One wave per right-hand side: the lanes stage the column and the rotations
// in LDS, lane 0 applies the rotations in order, the lanes write back.
constexpr int GW = 4;  // right-hand sides (waves) per work-group

__global__ void __launch_bounds__(64 * GW) k_gmres_step(int q, int j, int m, c128* __restrict__ H,
                                                        const c128* __restrict__ h1, const c128* __restrict__ h2,
                                                        const double* __restrict__ hnext, c128* __restrict__ cs,
                                                        c128* __restrict__ sn, c128* __restrict__ g,
                                                        double* __restrict__ est, int* __restrict__ st,
                                                        const double* __restrict__ thr, int maxit) {
  __shared__ double2 col_s[GW][128], cs_s[GW][128], sn_s[GW][128];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * GW + wv;
  if (b >= q) return;
  int* active = st;
  int* jdone = st + q;
  int* iters = st + 2 * q;
  if (!active[b]) return;
  c128* Hb = H + (long long)b * (m + 1) * m;
  c128* cb = cs + (long long)b * m;
  c128* sb = sn + (long long)b * m;
  c128* gb = g + (long long)b * (m + 1);
  c128* col = Hb + (long long)(m + 1) * j;
  double2* cl = col_s[wv];
  for (int t = lane; t <= j + 1; t += 64) {
    cl[t] = t <= j ? cadd(h1[t * q + b], h2[t * q + b]) : mk(hnext[b], 0.0);
    if (t < j) {
      cs_s[wv][t] = cb[t];
      sn_s[wv][t] = sb[t];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane == 0) {
    for (int t = 0; t < j; ++t) {
      const double2 a = cl[t], bb = cl[t + 1], c = cs_s[wv][t], s = sn_s[wv][t];
      cl[t] = cadd(cmulc(c, a), cmulc(s, bb));
      cl[t + 1] = csub(cmul(c, bb), cmul(s, a));
    }
    const double2 a = cl[j], bb = cl[j + 1];
    const double den = sqrt(cabs2(a) + cabs2(bb));
    double2 c, s;
    if (den == 0.0) {
      c = mk(1.0, 0.0);
      s = mk(0.0, 0.0);
    } else {
      c = cscale(a, 1.0 / den);
      s = cscale(bb, 1.0 / den);
    }
    cb[j] = c;
    sb[j] = s;
    cl[j] = mk(den, 0.0);
    cl[j + 1] = mk(0.0, 0.0);
    const double2 gj = gb[j];
    gb[j + 1] = mk(-(s.x * gj.x - s.y * gj.y), -(s.x * gj.y + s.y * gj.x));
    gb[j] = cmulc(c, gj);
    const double e = sqrt(cabs2(gb[j + 1]));
    est[b] = e;
    jdone[b] = j + 1;
    const int it = iters[b] + 1;
    iters[b] = it;
    if (e < thr[b] || it >= maxit) active[b] = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int t = lane; t <= j + 1; t += 64) col[t] = cl[t];
}

// any[0] = number of active right-hand sides
__global__ void k_count_active(int q, const int* __restrict__ st, int* __restrict__ any) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < q; b += blockDim.x)
    if (st[b]) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) any[0] = cnt;
}

// y[k*q + b] for k < jdone[b]: back substitution with the rotated (upper
// triangular) Hessenberg matrix.
__global__ void k_gmres_solve_small(int q, int m, const int* __restrict__ jdone, const c128* __restrict__ H,
                                    const c128* __restrict__ g, c128* __restrict__ y) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= q) return;
  const int jd = jdone[b];
  const c128* Hb = H + (long long)b * (m + 1) * m;
  const c128* gb = g + (long long)b * (m + 1);
  for (int k = jd - 1; k >= 0; --k) {
    double2 s = gb[k];
    for (int t = k + 1; t < jd; ++t) s = csub(s, cmul(Hb[(long long)(m + 1) * t + k], y[t * q + b]));
    y[k * q + b] = cdiv(s, Hb[(long long)(m + 1) * k + k]);
  }
  for (int k = jd; k < m; ++k) y[k * q + b] = mk(0.0, 0.0);
}

// u[b] += sum_{k < jdone[b]} Z_k[b] y[k][b]
__global__ void __launch_bounds__(TB) k_basis_combine(SegDev sg, const int* __restrict__ jdone,
                                                      const c128* __restrict__ Z, long long zstride,
                                                      const c128* __restrict__ y, c128* __restrict__ u) {
  const Chunk ch = chunk_of(sg, blockIdx.x);
  const int b = ch.b, S = sg.S;
  const int jd = jdone[b];
  if (jd == 0) return;
  for (long long i = ch.off + ch.lo + threadIdx.x; i < ch.off + ch.hi; i += TB) {
    double2 acc = u[i];
    for (int k = 0; k < jd; ++k) acc = cfma(Z[k * zstride + i], y[k * S + b], acc);
    u[i] = acc;
  }
}

// y[b] += x[b] for the systems with active[b] (active may be null)
__global__ void __launch_bounds__(TB) k_seg_add(SegDev sg, const int* __restrict__ active,
                                                const c128* __restrict__ x, c128* __restrict__ y) {
  const Chunk ch = chunk_of(sg, blockIdx.x);
  if (active && !active[ch.b]) return;
  for (long long i = ch.off + ch.lo + threadIdx.x; i < ch.off + ch.hi; i += TB) y[i] = cadd(y[i], x[i]);
}


}  // namespace

int multidot_nblocks(long long n) { return nblocks(n); }

hipError_t launch_multidot(int nk, const SegDev& sg, const c128* V, long long vstride, const c128* W,
                           c128* partial, c128* out, hipStream_t s, int wnorm, const int* skip) {
  if (nk <= 0 || sg.S <= 0) return hipSuccess;
  const int nkq = (nk + (wnorm ? 1 : 0)) * sg.S;
  const long long nlog = (long long)sg.G * ((nk + KG - 1) / KG);
  if (nlog > (1LL << 30)) return hipErrorInvalidValue;
  const long long grid = (nlog + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)grid), dim3(TB), 0, s, nk, sg, nkq, V, vstride, W, partial, wnorm,
                     skip);
  hipLaunchKernelGGL(k_dot_final, dim3((nkq + 63) / 64), dim3(64 * DF_SEG), 0, s, nkq, sg.S, sg.nb, partial, out,
                     skip);
  return hipGetLastError();
}

hipError_t launch_basis_update(int nk, const SegDev& sg, const c128* V, long long vstride, const c128* h, c128* W,
                               c128* partial, c128* nrm2, hipStream_t s, const int* skip) {
  if (nk <= 0 || sg.S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_basis_update, dim3(sg.G), dim3(TB), 0, s, nk, sg, V, vstride, h, W, nrm2 ? partial : nullptr,
                     skip);
  if (nrm2)
    hipLaunchKernelGGL(k_dot_final, dim3((sg.S + 63) / 64), dim3(64 * DF_SEG), 0, s, sg.S, sg.S, sg.nb, partial,
                       nrm2, skip);
  return hipGetLastError();
}

hipError_t launch_reorth_flag(int q, int nk, const c128* w0n2, const c128* w1n2, double eta, int* need, c128* h2,
                              hipStream_t s, const int* active) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reorth_flag, dim3((q + 127) / 128), dim3(128), 0, s, q, nk, w0n2, w1n2, eta * eta, need, h2,
                     active);
  return hipGetLastError();
}

hipError_t launch_normalize(const SegDev& sg, const c128* nrm2, const c128* x, c128* y, double* nrm, hipStream_t s,
                            const int* skip) {
  if (sg.S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize, dim3(sg.G), dim3(TB), 0, s, sg, nrm2, x, y, nrm, skip);
  return hipGetLastError();
}

hipError_t launch_seg_add(const SegDev& sg, const int* active, const c128* x, c128* y, hipStream_t s) {
  if (sg.S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_add, dim3(sg.G), dim3(TB), 0, s, sg, active, x, y);
  return hipGetLastError();
}

hipError_t launch_gmres_step(int q, int j, int m, c128* H, const c128* h1, const c128* h2, const double* hnext,
                             c128* cs, c128* sn, c128* g, double* est, int* state, const double* thr, int maxit,
                             int* any, hipStream_t s) {
  if (q <= 0) return hipSuccess;
  if (m > 126) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gmres_step, dim3((q + GW - 1) / GW), dim3(64 * GW), 0, s, q, j, m, H, h1, h2, hnext, cs, sn, g,
                     est, state, thr, maxit);
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, q, state, any);
  return hipGetLastError();
}

hipError_t launch_gmres_solve_small(int q, int m, const int* jdone, const c128* H, const c128* g, c128* y,
                                    hipStream_t s) {
  if (q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gmres_solve_small, dim3((q + 63) / 64), dim3(64), 0, s, q, m, jdone, H, g, y);
  return hipGetLastError();
}

hipError_t launch_basis_combine(const SegDev& sg, const int* jdone, const c128* Z, long long zstride, const c128* y,
                                c128* u, hipStream_t s) {
  if (sg.S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_basis_combine, dim3(sg.G), dim3(TB), 0, s, sg, jdone, Z, zstride, y, u);
  return hipGetLastError();
}
