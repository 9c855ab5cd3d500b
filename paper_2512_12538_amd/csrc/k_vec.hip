// Stencil application, restriction/prolongation between levels, and vector
// utilities.  All of these are bandwidth-bound streams over level buffers:
// one thread per node, consecutive threads on consecutive q (contiguous in
// memory), the grid's y dimension enumerating (box, column).
#include "kernels.h"

namespace {

constexpr int TB = 256;

// y = A_box x (mode 0) or y = b - A_box x (mode 1): one thread per node of a
// box, its five stencil coefficients formed once and applied to QG columns.
// The grid is one-dimensional and XCD-aware: the hardware places block i on
// XCD i mod 8, and logical block (i mod 8) * (gridDim.x / 8) + i / 8 makes
// every XCD run a contiguous range of node blocks, so the rows above and below
// a block (read by its stencil) sit in the same L2 as the block that loads
// them first.  Logical order: node block fastest, then box, then column group.
constexpr int QG = 2;
constexpr int NXCD = 8;

__global__ void __launch_bounds__(TB) k_apply_box(const OpDev* __restrict__ ops, const BoxDev* __restrict__ boxes, int nbox, int gxb,
                                                  int nlog, int q, const c128* __restrict__ x,
                                                  const c128* __restrict__ b, c128* __restrict__ y, int mode,
                                                  const int* __restrict__ active) {
  const int lb = (blockIdx.x % NXCD) * (gridDim.x / NXCD) + blockIdx.x / NXCD;
  if (lb >= nlog) return;
  const int nb = lb % gxb, t = lb / gxb;
  const int box = t % nbox, cg = t / nbox;
  const BoxDev B = boxes[box];
  const int c0 = cg * QG, c1 = c0 + QG < q ? c0 + QG : q;
  if (active) {
    bool any = false;
    for (int col = c0; col < c1; ++col) any = any || active[B.prob * q + col];
    if (!any) return;
  }
  const OpDev op = ops[B.prob];
  const int l = nb * TB + threadIdx.x;
  if (l >= B.n) return;
  const int a = l / B.ny, c = l - a * B.ny;
  const int p = B.p0 + a, qq = B.q0 + c;
  const double2 z = mk(0.0, 0.0);
  const double2 cd = stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, 0, 0);
  const bool hw = a > 0, he = a < B.nx - 1, hs = op.dim == 2 && c > 0, hn = op.dim == 2 && c < B.ny - 1;
  const double2 cw = hw ? stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, -1, 0) : z;
  const double2 ce = he ? stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, 1, 0) : z;
  const double2 cs = hs ? stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, 0, -1) : z;
  const double2 cn = hn ? stencil_coef(op, B.p0, B.p1, B.q0, B.q1, p, qq, 0, 1) : z;
  // absent neighbours read the node itself with a zero coefficient
  const int lw = hw ? l - B.ny : l, le = he ? l + B.ny : l, ls = hs ? l - 1 : l, ln = hn ? l + 1 : l;
#pragma unroll
  for (int col = c0; col < c1; ++col) {
    const c128* xb = x + B.voff * q + (long long)col * B.n;
    double2 v = cmul(cd, xb[l]);
    v = cfma(cw, xb[lw], v);
    v = cfma(ce, xb[le], v);
    v = cfma(cs, xb[ls], v);
    v = cfma(cn, xb[ln], v);
    const long long at = B.voff * q + (long long)col * B.n + l;
    if (mode == 1) v = csub(b[at], v);
    y[at] = v;
  }
}

__global__ void __launch_bounds__(TB) k_gather_children(const BoxDev* __restrict__ child,
                                                        const BoxDev* __restrict__ par, int q,
                                                        const c128* __restrict__ pbuf, c128* __restrict__ cbuf) {
  const int bc = blockIdx.y;
  const int box = bc / q, col = bc % q;
  const BoxDev C = child[box];
  const BoxDev P = par[C.parent];
  const long long cb = C.voff * q + (long long)col * C.n;
  const long long pb = P.voff * q + (long long)col * P.n;
  const int da = C.p0 - P.p0, dc = C.q0 - P.q0;
  for (int l = blockIdx.x * TB + threadIdx.x; l < C.n; l += gridDim.x * TB) {
    const int a = l / C.ny, c = l - a * C.ny;
    cbuf[cb + l] = pbuf[pb + (long long)(a + da) * P.ny + (c + dc)];
  }
}

__global__ void __launch_bounds__(TB) k_scatter_owned(const BoxDev* __restrict__ child,
                                                      const BoxDev* __restrict__ par, int q,
                                                      const c128* __restrict__ cbuf, c128* __restrict__ pbuf) {
  const int bc = blockIdx.y;
  const int box = bc / q, col = bc % q;
  const BoxDev C = child[box];
  const BoxDev P = par[C.parent];
  const long long cb = C.voff * q + (long long)col * C.n;
  const long long pb = P.voff * q + (long long)col * P.n;
  for (int t = blockIdx.x * TB + threadIdx.x; t < C.n_own; t += gridDim.x * TB) {
    const int oa = t / C.own_ny, oc = t - oa * C.own_ny;
    const int p = C.op0 + oa, qq = C.oq0 + oc;
    pbuf[pb + (long long)(p - P.p0) * P.ny + (qq - P.q0)] = cbuf[cb + (long long)(p - C.p0) * C.ny + (qq - C.q0)];
  }
}

__global__ void k_fill_zero(uint4* __restrict__ p, long long n16) {
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n16; i += (long long)gridDim.x * TB)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_fill_zero_bytes(unsigned char* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) p[i] = 0;
}

__global__ void k_copy(const c128* __restrict__ x, c128* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) y[i] = x[i];
}

__global__ void k_add_masked(const c128* __restrict__ x, c128* __restrict__ y, long long n,
                             const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const long long base = (long long)col * n;
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB)
    y[base + i] = cadd(y[base + i], x[base + i]);
}

__global__ void k_f64_to_f32(const c128* __restrict__ x, c64* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB)
    y[i] = to_c64(x[i]);
}

__global__ void __launch_bounds__(TB) k_rhs_g(const OpDev* __restrict__ ops, const BoxDev* __restrict__ root, int q,
                                              const c128* __restrict__ f, const c128* __restrict__ g,
                                              c128* __restrict__ out) {
  const BoxDev B = root[blockIdx.y / q];
  const OpDev op = ops[B.prob];
  const int col = blockIdx.y % q;
  const long long base = B.voff * q + (long long)col * B.n;
  for (int l = blockIdx.x * TB + threadIdx.x; l < B.n; l += gridDim.x * TB) {
    const int a = l / B.ny, c = l - a * B.ny;
    const int p = B.p0 + a, qq = B.q0 + c;
    const double cx = (double)((p > B.p0) + (p < B.p1));
    const double cy = op.dim == 2 ? (double)((qq > B.q0) + (qq < B.q1)) : 2.0;
    double nb = (p == B.p0 || p == B.p1) ? cy : 0.0;
    if (op.dim == 2 && (qq == B.q0 || qq == B.q1)) nb += cx;
    out[base + l] = cadd(f[base + l], cscale(g[base + l], 0.5 * nb / op.h));
  }
}

inline int grid_for(long long n, int cap = 4096) {
  long long g = (n + TB - 1) / TB;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_apply_box(const OpDev* ops, const BoxDev* boxes, int nbox, int max_n, int q,
                            const c128* x, const c128* b, c128* y, int mode, hipStream_t s, const int* active) {
  if (nbox <= 0 || q <= 0 || max_n <= 0) return hipSuccess;
  const int gxb = (max_n + TB - 1) / TB;
  const long long nlog = (long long)gxb * nbox * ((q + QG - 1) / QG);
  if (nlog > (1LL << 30)) return hipErrorInvalidValue;
  const long long grid = (nlog + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL(k_apply_box, dim3((unsigned)grid), dim3(TB), 0, s, ops, boxes, nbox, gxb, (int)nlog, q, x, b, y,
                     mode, active);
  return hipGetLastError();
}

hipError_t launch_gather_children(const BoxDev* child, int nchild, int max_n, const BoxDev* par, int q,
                                  const c128* pbuf, c128* cbuf, hipStream_t s) {
  if (nchild <= 0 || q <= 0) return hipSuccess;
  dim3 grid(grid_for(max_n, 1024), nchild * q);
  hipLaunchKernelGGL(k_gather_children, grid, dim3(TB), 0, s, child, par, q, pbuf, cbuf);
  return hipGetLastError();
}

hipError_t launch_scatter_owned(const BoxDev* child, int nchild, int max_own, const BoxDev* par, int q,
                                const c128* cbuf, c128* pbuf, hipStream_t s) {
  if (nchild <= 0 || q <= 0) return hipSuccess;
  dim3 grid(grid_for(max_own, 1024), nchild * q);
  hipLaunchKernelGGL(k_scatter_owned, grid, dim3(TB), 0, s, child, par, q, cbuf, pbuf);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && (bytes & 15) == 0) {
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(bytes / 16)), dim3(TB), 0, s, (uint4*)p, bytes / 16);
  } else {
    hipLaunchKernelGGL(k_fill_zero_bytes, dim3(grid_for(bytes)), dim3(TB), 0, s, (unsigned char*)p, bytes);
  }
  return hipGetLastError();
}

hipError_t launch_copy(const c128* x, c128* y, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(TB), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_add_masked(const c128* x, c128* y, long long n, int q, const int* active, hipStream_t s) {
  if (n <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_masked, dim3(grid_for(n, 1024), q), dim3(TB), 0, s, x, y, n, active);
  return hipGetLastError();
}

hipError_t launch_rhs_with_impedance(const OpDev* ops, const BoxDev* root, int nroot, int q, const c128* f, const c128* g,
                                     c128* out, hipStream_t s) {
  if (q <= 0 || nroot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs_g, dim3(1024, nroot * q), dim3(TB), 0, s, ops, root, q, f, g, out);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const c128* x, c64* y, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(TB), 0, s, x, y, n);
  return hipGetLastError();
}
