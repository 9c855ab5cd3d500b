/*
 * helmdd.h - C ABI of the hierarchical ORAS solver with randomised-SVD coarse
 * spaces for the impedance Helmholtz problem (MI355X / gfx950).
 *
 * Method (Gander, Jiang, Zhang, "Hierarchical Coarse Basis by Randomised SVD:
 * the Helmholtz Problem"):
 *   - problem: -u'' - k^2 u = f with impedance conditions d_n u - i k u = g
 *     (eq. (lap1), Sec. 1; in 2D the free-space problem of Sec. 3.1), here
 *     discretised by the cell-assembled 5-point (1D: 3-point) scheme on
 *     (N+1)^dim nodes, h = 1/N;
 *   - one step: ORAS smoothing u~ = u + sum_i P_i A~_i^{-1} R_i (f - A u)
 *     (eq. (sub1), Richardson form) followed by the coarse correction
 *     u = u~ + C A_c^{-1} C^H (f - A u~), A_c = C^H A C (eq. (coarse1));
 *   - coarse basis C = (C_i), C_i = P_i A~_i^{-1} B_i^T V_i with V_i the
 *     dominant right singular vectors of the interface map
 *     T_i = B_i^o A~_i^{-1} B_i^T, found by a randomised SVD (Sec. 2);
 *   - hierarchy: each subdomain problem is itself solved by n_i steps of the
 *     same two-level method on its children (Sec. 1, Sec. 2, Sec. 3 notation
 *     [m_x1 x m_y1, ...], n_c, n_i).
 *
 * Conventions
 *   - Every call returns hh_status; nothing throws across the boundary.
 *   - Complex numbers are interleaved (re, im) doubles ("c128").
 *   - Node (p, q), 0 <= p, q <= N, has index p*(N+1) + q (1D: index p).
 *   - Device pointers are HIP device memory owned by the caller; the library
 *     never frees them.  The context owns every internal allocation
 *     (factorisations, coarse bases, A_c^{-1}, work space) until hh_destroy,
 *     which returns it to a process-wide cache of device blocks that later
 *     contexts reuse (hh_release_cached_memory frees the cache).
 *   - All device work is enqueued on hh_options.stream (null: the default
 *     stream), which must stay valid until hh_destroy returns.  Calls return
 *     after the work they started has completed, except where stated.  A
 *     context is used by one host thread at a time; separate contexts may be
 *     used concurrently from separate threads and streams.
 *   - On HH_EDEVICE the context is poisoned: only hh_destroy is valid.
 */
#ifndef HELMDD_H
#define HELMDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HH_OK = 0,
  HH_EINVAL = 1,       /* invalid argument or shape; no side effect */
  HH_ENOMEM = 2,       /* device allocation failed; context unchanged */
  HH_EDEVICE = 3,      /* HIP error; context poisoned */
  HH_ENOTCONV = 4,     /* outer loop hit maxit; u holds the last iterate */
  HH_ESINGULAR = 5,    /* zero pivot in a leaf factorisation or in A_c */
  HH_ESTATE = 6,       /* call out of order (e.g. solve before the coarse build) */
  HH_EUNSUPPORTED = 7  /* valid but not implemented (size limits below) */
} hh_status;

typedef enum { HH_FP64 = 0, HH_MIXED = 1 } hh_precision;
typedef enum { HH_STATIONARY = 0, HH_GMRES = 1 } hh_outer;

typedef struct hh_ctx hh_ctx; /* opaque */

/* The operator of eq. (lap1) / Sec. 3.1: dim 1 or 2, N cells per side,
 * wavenumber per node (host array of (N+1)^dim doubles, copied by hh_setup)
 * or the constant k_const when k is null. */
typedef struct {
  int32_t dim;
  int32_t n_cells;
  const double* k;
  double k_const;
} hh_operator;

/* The decomposition [m_x1 x m_y1, ..., m_xl x m_yl] of Sec. 3: level l splits
 * every box of level l-1 into m[l-1][0] x m[l-1][1] boxes (1D: m[l-1][1] is
 * ignored).  overlap_cells[l-1] = delta/h (even): each box is extended by
 * delta/(2h) cells on every side interior to its parent.  inner_iters[l-1] =
 * n_i, the number of two-level steps that solve a level-l box problem when
 * the box has children (default 1 when 0). */
typedef struct {
  int32_t levels;
  int32_t m[8][2];
  int32_t overlap_cells[8];
  int32_t inner_iters[8];
} hh_decomposition;

typedef struct {
  int32_t precision;     /* hh_precision: HH_MIXED keeps the leaf factors in complex64 */
  int32_t outer;         /* hh_outer used by hh_solve */
  int32_t gmres_restart; /* restart length (default 50 when <= 0, at most 120) */
  int32_t full_reorth;   /* GMRES Arnoldi: 1 = classical Gram-Schmidt twice at every step;
                            0 = second pass only where the first cancelled ||w|| by more than 8x */
  void* stream;          /* hipStream_t, or null */
  int32_t autotune;      /* 1: on the first solve with a given nrhs, time the leaf sweep with 1, 2 and 4
                            right-hand sides per work-group for every leaf shape and keep the fastest
                            (the arithmetic of a column does not depend on it) */
  int32_t graphs;        /* 1: from the second GMRES solve with a given nrhs on, each Arnoldi step is
                            captured once into a HIP graph and replayed (stream must not be null);
                            results are bit-identical to the eager steps */
} hh_options;

typedef struct {
  int32_t iters;        /* preconditioner applications */
  int32_t converged;    /* 1 if ||f - A u|| / ||f|| < rtol */
  double rel_residual;  /* true relative residual at exit */
} hh_solve_info;

/* Builds the decomposition, uploads k and factorises every leaf box problem
 * A~_i (local impedance conditions, eq. (sub1)) on the device.  Leaf boxes must
 * have at most 256 nodes along q.  HH_ESINGULAR if a leaf factorisation meets a
 * zero pivot. */
hh_status hh_setup(const hh_operator* A, const hh_decomposition* d, const hh_options* o, hh_ctx** out);

/* Independent problems in one context (the local problems of every level of
 * every problem go into the same launches).  A[p], d[p] (p < nprob): operator
 * and decomposition of problem p; all problems share dim and the number of
 * levels.  The boxes of a level are numbered problem by problem, so per-box
 * arrays of the other calls (hh_level_info, omega of hh_build_coarse) list
 * problem 0's boxes first.  Whole-domain vectors of the other calls hold, per
 * problem in order, its nrhs columns: [p][nrhs][n_p] with n_p = (N_p+1)^dim
 * (hh_problem_layout gives the offsets); hh_solve's info has nprob * nrhs
 * entries, problem-major.  Same errors as hh_setup (HH_EINVAL also when the
 * problems differ in dim or depth).  hh_setup is hh_setup_batch with nprob = 1. */
hh_status hh_setup_batch(int32_t nprob, const hh_operator* A, const hh_decomposition* d, const hh_options* o,
                         hh_ctx** out);

/* The leaf sweep plan: the leaves grouped by shape bucket (0..5: widths up
 * to 8, 16, 40, 72, 144, 256 nodes), per group its bucket, leaf count, widest
 * leaf, and the right-hand sides per work-group the autotuner chose (qb) for
 * nrhs = tuned_for (0 when not tuned: chosen from the launch size).  Arrays
 * have ngroups entries (at most 6); any may be null. */
hh_status hh_sweep_plan(const hh_ctx* c, int32_t* ngroups, int32_t* bucket, int32_t* count, int32_t* max_width,
                        int32_t* qb, int32_t* tuned_for);

/* nprob, and per problem its node count n_p and the offset (in complex entries,
 * per right-hand side) of its block: problem p's column c starts at
 * nrhs * offset[p] + c * n_p.  Arrays have nprob entries; any may be null. */
hh_status hh_problem_layout(const hh_ctx* c, int32_t* nprob, int64_t* n_nodes, int64_t* offset);

/* Number of boxes of a level (0 = the whole domain) and, per box, its interface
 * size m_in, coarse rank r_i = min(rank_per_interface * n_if, m_in) and sketch
 * width s_i = min(r_i + oversample, m_in) (n_if = interface sides of the box).
 * Arrays have n_boxes entries; any of them may be null. */
hh_status hh_level_info(const hh_ctx* c, int32_t level, int32_t rank_per_interface, int32_t oversample,
                        int32_t* n_boxes, int32_t* m_in, int32_t* r, int32_t* s);

/* Randomised SVD of every interface map of `level` and the coarse spaces of
 * the parents at level-1 (Sec. 2): Y = T_i Omega_i, Q = qr(Y),
 * B^H = T_i^* Q, V_i = top-r_i right singular vectors of B,
 * C_i = P_i S_i(B_i^T V_i), A_c = C^H A C and A_c^{-1} (FP64, partial pivoting).
 * Must be called for level L, L-1, ..., 1 in this order (an upper level's
 * sub-solves use the coarse spaces below it), else HH_ESTATE.
 * omega: device c128, the Gaussian blocks of the level's boxes concatenated in
 * box order, block i column-major m_in x s_i (sample t = column t); null is
 * valid only when rank_per_interface == 0 (no coarse space at this level). */
hh_status hh_build_coarse(hh_ctx* c, int32_t level, int32_t rank_per_interface, int32_t oversample,
                          const void* omega);

/* Solves A u = b for nrhs right-hand sides: b = f + impedance data g (2D:
 * (boundary edges at the node)/2 * g/h, 1D: g/h at the end nodes).
 * f, g, u: device c128 arrays [nrhs][(N+1)^dim] (a batch: per problem, see
 * hh_setup_batch); g may be null (g = 0).
 * u0 = 0; the outer loop (hh_options.outer) stops when
 * ||b - A u||_2 / ||b||_2 < rtol or after maxit preconditioner applications
 * (rtol = 0 runs exactly maxit).  info: host array of nrhs entries (a batch:
 * nprob * nrhs) or null.
 * HH_ENOTCONV if some right-hand side did not converge. */
hh_status hh_solve(hh_ctx* c, int32_t nrhs, const void* f, const void* g, void* u, double rtol, int32_t maxit,
                   hh_solve_info* info);

/* y = A x (mode 0) or y = b - A x (mode 1, b device c128) for nrhs vectors of
 * the whole-domain operator.  Device c128 [nrhs][(N+1)^dim]. */
hh_status hh_apply_operator(hh_ctx* c, int32_t nrhs, const void* x, const void* b, void* y, int32_t mode);

/* z = B(r): one two-level step of eqs. (sub1)-(coarse1) from zero, including
 * the hierarchy below.  Device c128 [nrhs][(N+1)^dim]. */
hh_status hh_precondition(hh_ctx* c, int32_t nrhs, const void* r, void* z);

/* Copies out the coarse data of parent box `parent` at level `level` (the
 * parent's children are the boxes of level+1): n_c (host int), and when the
 * pointers are non-null, A_c (host c128, n_c x n_c column-major), and the
 * singular values of the sketch of each child (host doubles, s_i per child in
 * child order).  A_c is returned before inversion. */
hh_status hh_get_coarse(hh_ctx* c, int32_t level, int32_t parent, int32_t* n_c, void* Ac_host, double* sigma_host);

/* Copies out the coarse block C_i of box i of level `level` (children of some
 * parent at level-1) on the box's owned nodes: host c128, r_i columns of
 * n_own entries (owned box p-major).  n_own and r_i returned when non-null. */
hh_status hh_get_basis(hh_ctx* c, int32_t level, int32_t box, int32_t* n_own, int32_t* r_i, void* C_host);

/* Live kernel timing.  hh_profile(c, 1) clears the counters and brackets every
 * later launch of the profiled kernel families with HIP events on the
 * context's stream; hh_profile(c, 0) stops.  hh_profile_read returns, for a
 * family, the number of launches, their summed event time (ms), and the
 * summed algorithmic bytes and flops of those launches:
 *   family 0  leaf block-tridiagonal solve (every G_j streamed once per sweep,
 *             right-hand side and solution vectors: bytes = sum over leaves of
 *             (2 nx - 1) b^2 e + 64 q n_i, flops = 8 (2 nx - 1) b^2 q;
 *             e = 16 bytes for complex128 factors, 8 for complex64)
 *   family 1  first Gram-Schmidt update W -= V h (bytes 16 n q (j + 3))
 *   family 2  first Gram-Schmidt inner products V^H W (bytes 16 n q (j + 1 + ceil(j / 8)))
 *   family 3  5-point stencil y = A z of every Arnoldi step (eq. (lap1); bytes
 *             32 n q: z read and y written once, coefficients from (h, k) in
 *             registers; flops 40 n q)
 * Profiling inserts events between launches; leave it off for timing runs. */
hh_status hh_profile(hh_ctx* c, int32_t enable);
hh_status hh_profile_read(hh_ctx* c, int32_t family, int64_t* launches, double* total_ms, double* bytes,
                          double* flops);

hh_status hh_destroy(hh_ctx* c);

/* ------------------------------------------------------------------ serving
 * A server solves requests for many operators on one GPU: worker threads,
 * each with its own HIP stream, take the oldest queued request whose operator
 * is idle together with the other queued requests for that operator and
 * tolerance (up to max_batch_rhs right-hand sides) and run them as one
 * hh_solve.  Prepared operators (leaf factors and the coarse spaces of all
 * levels, built with Gaussian blocks drawn by hh_omega_philox from the
 * request's seed) stay on the device, keyed by operator_id.  A new operator
 * is admitted when its estimated footprint plus the batch's work space fits
 * budget_bytes, after idle operators are evicted least-recently-used first;
 * otherwise it waits for running batches to end (HH_ENOMEM if it cannot fit
 * even alone).  Every right-hand side gives the same result in any batch.
 * Thread-safe: any thread may submit and wait. */
typedef struct hh_server hh_server;

typedef struct {
  int64_t budget_bytes;  /* device bytes for prepared operators and running batches */
  int32_t workers;       /* batches in flight, 1..16 (one stream each) */
  int32_t max_batch_rhs; /* right-hand sides per batch (and per request), >= 1 */
  int32_t precision;     /* hh_precision of every operator */
  int32_t gmres_restart; /* 0: 50 */
} hh_server_options;

typedef struct {
  uint64_t operator_id;           /* one id, one (operator, decomposition, ranks, seed) */
  hh_operator op;                 /* k (host) copied at the first request of an id */
  hh_decomposition decomposition;
  int32_t rank_per_interface[8];  /* per level l at index l-1; 0: no coarse space there */
  int32_t oversample;
  uint64_t omega_seed;
  int32_t nrhs;
  const void* f;                  /* device c128 [nrhs][(N+1)^dim], valid until completion */
  void* u;                        /* device c128 [nrhs][(N+1)^dim], written at completion */
  double rtol;                    /* as hh_solve; batched only with equal rtol and maxit */
  int32_t maxit;
} hh_request;

typedef struct {
  int32_t status;       /* hh_status of the request (HH_ENOTCONV: some rhs missed rtol) */
  int32_t iters;        /* largest preconditioner-application count over its rhs */
  double rel_residual;  /* largest true relative residual over its rhs */
  double latency_s;     /* submit to result in u (its stream synchronised) */
  double queue_s;       /* submit to the start of its batch */
  int32_t batch_rhs;    /* right-hand sides of the batch that carried it */
  int32_t cache_hit;    /* 1 if its operator was already prepared */
} hh_request_result;

hh_status hh_server_create(const hh_server_options* o, hh_server** out);
/* Queues a request; *ticket identifies it.  HH_EINVAL for an invalid request
 * or an id reused with another shape.  f and u must be ready when the call is
 * made: the server's own streams do not wait for work queued elsewhere, so any
 * pending write to f or u (a fill of u included) must have completed.  u is
 * written once, before the result is handed out by hh_server_wait. */
hh_status hh_server_submit(hh_server* s, const hh_request* r, uint64_t* ticket);
/* Waits (timeout_s < 0: without limit) for the request; HH_ESTATE on timeout.
 * A completed ticket is released by the call that returns its result. */
hh_status hh_server_wait(hh_server* s, uint64_t ticket, double timeout_s, hh_request_result* res);
hh_status hh_server_stats(hh_server* s, int64_t* served, int64_t* misses, int64_t* evictions, int64_t* cached,
                          int64_t* reserved_bytes);
/* Message of the server's last failed batch (status, operator id, batch width
 * and the context's or set-up's error text), or "" when none failed.  The
 * pointer is valid on the calling thread until its next call of this function. */
const char* hh_server_last_error(hh_server* s);
/* Stops the workers after their running batches; queued requests are dropped. */
hh_status hh_server_destroy(hh_server* s);

/* Host-side estimate of the peak device bytes of setting up an operator and
 * solving with nrhs right-hand sides: the prepared operator plus the larger of
 * the set-up's transient work space and the solve's (what the server reserves
 * when it admits a new operator).  rank: per level, as in hh_request. */
hh_status hh_estimate_device_bytes(const hh_operator* A, const hh_decomposition* d, const int32_t* rank,
                                   int32_t oversample, int32_t nrhs, int32_t gmres_restart, int32_t precision,
                                   int64_t* bytes);

/* The Gaussian test block Omega of (level, box) the server draws from a seed:
 * s x m_in complex entries CN(0,1), row-major (sample t, node j), as
 * interleaved (re, im) doubles into out (host).  Philox4x32-10 with counter
 * (t * m_in + j, box, level, 0x4f4d4547) and key (seed low, high words); two
 * 53-bit uniforms per entry, Box-Muller. */
hh_status hh_omega_philox(uint64_t seed, int32_t level, int32_t box, int32_t m_in, int32_t s, double* out);

/* Frees the device blocks cached by the library on the current device (blocks
 * released by destroyed contexts and by buffer regrowth); *bytes (if non-null)
 * receives the amount freed.  The cache holds at most a quarter of the device
 * memory, or HH_POOL_CAP_GB gigabytes when that environment variable is set
 * (read at the first allocation on the device). */
hh_status hh_release_cached_memory(int64_t* bytes);
/* Message of the last failed call on context c; with c = NULL, the message of
 * the calling thread's last failed hh_setup / hh_setup_batch (whose context no
 * longer exists), or "null context".  The pointer stays valid until the next
 * call on c (or the next set-up on this thread). */
const char* hh_last_error(const hh_ctx* c);
const char* hh_status_string(hh_status s);

#ifdef __cplusplus
}
#endif

#endif /* HELMDD_H */
