// Launch wrappers of the HIP kernels.  Every wrapper enqueues on the given
// stream and returns hipGetLastError().  Level buffers hold, for each box of a
// level, q columns of the box's local vector: box i, column c, local node x at
// index voff_i * q + c * n_i + x.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

// ---------------------------------------------------------------- vectors / stencil (k_vec.hip)
// y = A_box x (mode 0) or y = b - A_box x (mode 1) for every box and column of a level buffer;
// with active (nprob * q flags) only the columns of active (problem, right-hand side) pairs.
hipError_t launch_apply_box(const OpDev* ops, const BoxDev* boxes, int nbox, int max_n, int q,
                            const c128* x, const c128* b, c128* y, int mode, hipStream_t s,
                            const int* active = nullptr);
// child[c][col][x] = parent[parent(c)][col][R_c x]
hipError_t launch_gather_children(const BoxDev* child, int nchild, int max_n, const BoxDev* par, int q,
                                  const c128* pbuf, c128* cbuf, hipStream_t s);
// parent[parent(c)][col][x] = child[c][col][x] for x owned by c
hipError_t launch_scatter_owned(const BoxDev* child, int nchild, int max_own, const BoxDev* par, int q,
                                const c128* cbuf, c128* pbuf, hipStream_t s);
hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t s);
hipError_t launch_copy(const c128* x, c128* y, long long n, hipStream_t s);
// y[col] += x[col] for the columns with active[col] != 0 (all if active is null); columns of length n
hipError_t launch_add_masked(const c128* x, c128* y, long long n, int q, const int* active, hipStream_t s);
hipError_t launch_f64_to_f32(const c128* x, c64* y, long long n, hipStream_t s);
// out = f + (boundary edges at the node)/2 * g / h on every whole-domain box (1D: g/h at the ends)
hipError_t launch_rhs_with_impedance(const OpDev* ops, const BoxDev* root, int nroot, int q, const c128* f, const c128* g,
                                     c128* out, hipStream_t s);

// ---------------------------------------------------------------- leaf solves (k_leaf.hip, k_sweep.hip)
// Two-ended block-tridiagonal factorisation of the leaf boxes lidx[0 .. count)
// of nleaf (FP64, widths at most max_ny): G_j per grid line, chains from both
// ends to the middle line nx / 2.  info: 3 nleaf ints (chains 2 leaf + half,
// then middle lines 2 nleaf + leaf); nonzero = first zero pivot.
hipError_t launch_leaf_factor(const OpDev* ops, const BoxDev* leaves, int nleaf, const int* lidx, int count,
                              int max_ny, c128* G, int* info, hipStream_t s);
// Factorisation kernel class of a leaf of width ny (0..6).
int leaf_factor_bucket(int ny);
// Sweep shape bucket of a leaf of width ny (0..5; -1: wider than 256).
int leaf_sweep_bucket(int ny);
// x = A~^{-1} rhs for the leaf boxes lidx[0 .. count) (all of one shape
// bucket) and q columns (two launches).  rhs and x are distinct level buffers;
// edge holds 2 nleaf * q * edge_ld entries of work space (edge_ld >= every
// leaf's width).  qb: right-hand sides per work-group (1, 2 or 4; 0 = chosen
// from the launch size); it does not change the arithmetic.  G (T = double:
// FP64 factors, float: complex64 copy) needs 65536 zero entries past the last
// leaf.  With par given, the right-hand side is read in place from the parent
// buffer (R_i r) and, with out given, the solution goes to the parent buffer on
// the owned nodes only (P_i x, every parent node owned by one leaf); x then
// serves as work space.  active (nullable, nprob * q flags): right-hand sides
// whose outputs are needed; a work-group whose columns are all inactive exits.
template <typename T>
hipError_t launch_leaf_solve(const OpDev* ops, const BoxDev* leaves, const int* lidx, int count, int bucket,
                             int edge_ld, int q, int qb, const typename cvec<T>::type* G, const c128* rhs, c128* x,
                             c128* edge, const BoxDev* par, c128* out, const int* active, hipStream_t s);

// ---------------------------------------------------------------- interface map / rSVD (k_rsvd.hip)
// buf[box][c][iface[t]] = vals[voff[box] + c*m_in + t] for c < (use_r ? r : s); buf pre-zeroed
hipError_t launch_iface_scatter(const BoxDev* boxes, int nbox, int q, const int* if_idx, const long long* voff,
                                const c128* vals, int use_r, c128* buf, hipStream_t s);
// vals[voff[box] + c*m_in + t] = buf[box][c][iface[t]] (conjugated with conj_in)
hipError_t launch_iface_gather(const BoxDev* boxes, int nbox, int q, const int* if_idx, const long long* voff,
                               const c128* buf, c128* vals, int use_r, int conj_in, hipStream_t s);
// Y[yoff[box] + c*tr_cnt + row] = (A~_j R_j P_i X)[x_row]
hipError_t launch_trace(const OpDev* ops, const BoxDev* boxes, int nbox, int q, const int2* rows,
                        const long long* yoff, const c128* X, c128* Y, hipStream_t s);
// H[box][c][y] = conj(sum_rows conj(A~_j[x, y]) Q[row][c]); H pre-zeroed
hipError_t launch_trace_adjoint(const OpDev* ops, const BoxDev* boxes, int nbox, int q, const int2* rows,
                                const int* seg_ptr, const int* seg_y, const int4* adj, const long long* yoff,
                                const c128* Qm, c128* H, hipStream_t s);
// Batched Householder QR: A[b] (m_b x n_b col-major) -> explicit Q in place, R (n_b x n_b); n_b <= 128
hipError_t launch_qr(int nprob, const int* m, const int* n, const long long* aoff, c128* A, const long long* roff,
                     c128* R, c128* work, hipStream_t s);
// One-sided Jacobi SVD of R[b] (n_b x n_b, n_b <= nmax <= 128): U sorted by decreasing singular value,
// sigma; the rotations run in shared memory when nmax <= 96 (R left as it was), else on R in place
hipError_t launch_jacobi_svd(int nprob, const int* n, int nmax, const long long* roff, c128* R,
                             const long long* uoff, c128* U, double* sigma, const long long* soff, hipStream_t s);
// V[b] (m_b x r_b) = Q[b] (m_b x n_b) * U[b][:, :r_b]
hipError_t launch_small_gemm(int nprob, int max_mr, const int* m, const int* n, const int* r, const long long* qoff,
                             const c128* Q, const long long* uoff, const c128* U, const long long* voff, c128* V,
                             hipStream_t s);
// C[box] (r x n_own) = buf[box][c][owned nodes]
hipError_t launch_extract_owned(const BoxDev* boxes, int nbox, int max_own, int q, const c128* buf, c128* C,
                                hipStream_t s);

// ---------------------------------------------------------------- coarse space (k_coarse.hip)
hipError_t launch_galerkin_ac(const OpDev* ops, const BoxDev* boxes, int nbox, const BoxDev* par, const int4* dil,
                              int max_dil, int rmax, const c128* C, c128* AC, hipStream_t s);
hipError_t launch_galerkin_blocks(const BoxDev* boxes, const ParentDev* pars, const int4* pairs, int npairs,
                                  int rmax, const int4* dil, const c128* C, const c128* AC, c128* Ac,
                                  hipStream_t s);
// Negligible coarse modes: a column of C_i whose norm on the owned nodes is at most tol
// times the box's largest is zeroed and flagged in drop[box * rmax + t] (rmax <= 128)
hipError_t launch_drop_negligible(const BoxDev* boxes, int nbox, int rmax, double tol, c128* C, int* drop,
                                  hipStream_t s);
// A_c diagonal entries of the dropped modes set to one (their rows and columns are zero)
hipError_t launch_unit_dropped(const BoxDev* boxes, const ParentDev* pd, int nbox, int rmax, const int* drop,
                               c128* A, hipStream_t s);
// In-place inverse of every parent's A_c (Gauss-Jordan, partial pivoting); piv and fcol hold
// npar*max_nc entries; info[p] = first zero pivot + 1 (0 if none)
hipError_t launch_gj_inverse(const ParentDev* pars, int npar, int max_nc, c128* A, int* piv, c128* fcol, int* info,
                             hipStream_t s);
// cvec[par][c][cidx + a] = C_child[a]^H t[par][c][owned nodes of child]: FP64
// matrix-core products over chunks of restrict_chunk_nodes() owned nodes into
// `part` (restrict_workspace(nchunks, rmax, q) entries), then an ordered sum
// over each child's chunks.  chunks[g] = (child, chunk index) for the chunks of
// every child with a coarse space, child-major; cbase[child] = its first chunk.
// active (nullable): flags per system (problem * q + column); results for
// inactive systems are left undefined, as in the leaf sweeps.
int restrict_chunk_nodes();
long long restrict_workspace(int nchunks, int rmax, int q);
hipError_t launch_coarse_restrict(const BoxDev* child, int nchild, const int2* chunks, const int* cbase, int nchunks,
                                  const BoxDev* par, const ParentDev* pd, int rmax, int q, const c128* C,
                                  const c128* t, c128* part, c128* cvec, const int* active, hipStream_t s);
// y[par][c] = A_c^{-1} cvec[par][c] (FP64 matrix cores)
hipError_t launch_coarse_gemv(const ParentDev* pd, int npar, int max_nc, int q, const c128* Ainv,
                              const c128* cvec, c128* y, hipStream_t s);
// u[par][c][owned nodes of child] += C_child y[par][c][cidx ..] (FP64 matrix cores);
// groups[g] = (child, group of prolong_group_nodes() owned nodes) for every child
// with a coarse space
int prolong_group_nodes();
hipError_t launch_coarse_prolong(const BoxDev* child, const int2* groups, int ngroups, int rmax, const BoxDev* par,
                                 const ParentDev* pd, int q, const c128* C, const c128* y, c128* u,
                                 const int* active, hipStream_t s);

// ---------------------------------------------------------------- Krylov (k_krylov.hip)
// The systems of the outer loop (one per problem and right-hand side): system
// b is the segment [off[b], off[b] + len[b]) of a level-0 vector.  Its
// reductions run over nb[b] = multidot_nblocks(len[b]) chunks; the chunks of
// all systems are numbered consecutively, chunk g = (system, index) = chunk[g].
struct SegDev {
  const long long* off = nullptr;
  const int* len = nullptr;
  const int* nb = nullptr;
  const int2* chunk = nullptr;
  int S = 0, G = 0, NBmax = 0;
};
int multidot_nblocks(long long n);
// out[k*S + b] = sum_x conj(V_k[b][x]) W[b][x], k < nk (V_k at V + k*vstride); with wnorm also
// out[nk*S + b] = |W[b]|^2; systems with skip[b] == 0 untouched (skip may be null);
// partial: (nk+1)*S*NBmax entries
hipError_t launch_multidot(int nk, const SegDev& sg, const c128* V, long long vstride, const c128* W,
                           c128* partial, c128* out, hipStream_t s, int wnorm = 0, const int* skip = nullptr);
// W[b] -= sum_k V_k[b] h[k*S + b]; if nrm2 is non-null also nrm2[b] = ||W[b]||^2 after the update
// (partial: S*NBmax scratch entries); systems with skip[b] == 0 untouched
hipError_t launch_basis_update(int nk, const SegDev& sg, const c128* V, long long vstride, const c128* h, c128* W,
                               c128* partial, c128* nrm2, hipStream_t s, const int* skip = nullptr);
// need[b] = active[b] and (w1n2[b] < eta^2 w0n2[b]) (always when eta >= 1; active may be null);
// h2[:, b] = 0 where not needed
hipError_t launch_reorth_flag(int q, int nk, const c128* w0n2, const c128* w1n2, double eta, int* need, c128* h2,
                              hipStream_t s, const int* active = nullptr);
// y[b] = x[b] / sqrt(re nrm2[b]) (zero if the norm is zero); nrm[b] = the norm; systems with
// skip[b] == 0 untouched (skip may be null)
hipError_t launch_normalize(const SegDev& sg, const c128* nrm2, const c128* x, c128* y, double* nrm, hipStream_t s,
                            const int* skip = nullptr);
// y[b] += x[b] for the systems with active[b] (active may be null)
hipError_t launch_seg_add(const SegDev& sg, const int* active, const c128* x, c128* y, hipStream_t s);
// GMRES column j for every active rhs; state = [active[q], jdone[q], iters[q]]; a rhs turns
// inactive when |g_{j+1}| < thr[b] or iters >= maxit; any[0] = number still active
hipError_t launch_gmres_step(int q, int j, int m, c128* H, const c128* h1, const c128* h2, const double* hnext,
                             c128* cs, c128* sn, c128* g, double* est, int* state, const double* thr, int maxit,
                             int* any, hipStream_t s);
hipError_t launch_gmres_solve_small(int q, int m, const int* jdone, const c128* H, const c128* g, c128* y,
                                    hipStream_t s);
// u[b] += sum_{k < jdone[b]} Z_k[b] y[k*S + b]
hipError_t launch_basis_combine(const SegDev& sg, const int* jdone, const c128* Z, long long zstride, const c128* y,
                                c128* u, hipStream_t s);
