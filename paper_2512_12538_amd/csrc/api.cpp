// C ABI and host orchestration of the hierarchical ORAS solver.
//
// The host only decides what runs: it builds the integer tables of the
// decomposition, sizes the device buffers and enqueues kernels; every
// floating-point step (factorisations, stencils, solves, QR, SVD, Galerkin
// products, inversions, Krylov updates) runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/helmdd.h"
#include "geometry.h"
#include "internal.h"
#include "kernels.h"
#include "pool.h"

namespace {

// A coarse mode whose extension P_i S_i(B_i^T v) has a norm on the owned nodes of at
// most this fraction of the largest of its box is not used (it would add a
// numerically zero column to C and make A_c singular).
constexpr double kNegligibleMode = 1e-10;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Leaves of one kernel shape: order[start .. start + count) of a level's
// leaf-order array, widths at most max_ny.
struct LeafGroup {
  int key = 0, start = 0, count = 0, max_ny = 0;
  int qb = 0, qb_q = 0;  // sweep: right-hand sides per work-group chosen for qb_q columns (0: not tuned)
};

struct Level {
  int nbox = 0;
  std::vector<BoxDev> hb;
  BoxDev* d = nullptr;
  long long total = 0;  // sum of box sizes
  int max_n = 0, max_nx = 0, max_ny = 0, max_own = 0;
  int* d_if = nullptr;
  std::vector<long long> if_off;  // per box
  // --- this level's boxes as children of a coarse space (built by build_coarse(level))
  bool built = false;
  int rank = 0, rmax = 0, smax = 0;
  bool tables = false;
  int2* d_rows = nullptr;
  int* d_seg_ptr = nullptr;
  int* d_seg_y = nullptr;
  int4* d_adj = nullptr;
  int max_tr = 0;
  c128* C = nullptr;
  c128* AC = nullptr;
  int4* d_dil = nullptr;
  int max_dil = 0;
  int4* d_pairs = nullptr;
  int npairs = 0;
  // work lists of the coarse restriction (chunks of owned nodes) and prolongation (node groups)
  int2* d_rchunks = nullptr;
  int* d_rcbase = nullptr;
  int n_rchunks = 0;
  int2* d_pgroups = nullptr;
  int n_pgroups = 0;
  std::vector<double> sigma;       // per box, smax entries
  // --- this level's boxes as parents (coarse space of their problems)
  std::vector<ParentDev> hp;
  ParentDev* dp = nullptr;
  int max_nc = 0;
  bool has_coarse = false;
  c128* Ainv = nullptr;
  c128* Araw = nullptr;
  int* d_piv = nullptr;
  long long nc_total = 0, nc2_total = 0;
  // --- work buffers, capacity qcap columns
  int qcap = 0;
  c128 *R = nullptr, *X = nullptr, *T = nullptr, *E = nullptr, *U = nullptr;
  c128 *cvec = nullptr, *yvec = nullptr;
  c128* W = nullptr;   // leaf level: the two half-sweep end lines per box (2 nbox q max_ny)
  c128* RP = nullptr;  // parent levels: chunk partial sums of the coarse restriction
  long long rp_len = 0;
  // leaf level: leaves grouped by sweep shape and by factorisation kernel
  std::vector<LeafGroup> sweep_groups, factor_groups;
  int *d_sweep_order = nullptr, *d_factor_order = nullptr;
};

}  // namespace

struct hh_ctx {
  std::string err;
  bool poisoned = false;
  hipStream_t stream = nullptr;
  int precision = HH_FP64;
  int outer = HH_GMRES;
  int restart = 50;
  double reorth_eta = 0.125;
  // outer-loop systems whose preconditioner outputs are needed (device flags,
  // nprob * q), set while GMRES iterates; null: all
  const int* act = nullptr;
  Geometry geo;             // all problems of the batch, merged level by level
  int nprob = 1;
  std::vector<OpDev> hops;  // per problem (k points into d_k)
  OpDev* d_ops = nullptr;
  double* d_k = nullptr;
  bool autotune = false;  // time the sweep's column-group widths on the first use of a q
  bool graphs = false;    // replay captured Arnoldi steps (from the second solve with a q on)
  bool capturing = false;
  int gw_maxit = -1;      // maxit the step graphs were captured with
  long long epoch = 0;    // bumped whenever a buffer or table used inside a captured step changes
  // persistent GMRES work space (the captured steps refer to it) and the step graphs
  struct Gmres {
    int q = 0, m = 0, solves = 0;
    long long epoch = -1;
    c128 *Vb = nullptr, *Zb = nullptr, *W = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
    c128 *h1 = nullptr, *h2 = nullptr, *tmp = nullptr, *y = nullptr;
    double *hn = nullptr, *est = nullptr, *thr = nullptr;
    int *state = nullptr, *any = nullptr, *need = nullptr;
    std::vector<hipGraphExec_t> exec;
  } gw;
  // outer-loop systems (problem, right-hand side) for sg_q right-hand sides
  SegDev sg;
  int sg_q = 0;
  long long* d_seg_off = nullptr;
  int *d_seg_len = nullptr, *d_seg_nb = nullptr;
  int2* d_seg_chunk = nullptr;
  int L = 0;
  std::vector<int> inner;
  std::vector<Level> lv;
  c128* G = nullptr;  // FP64 leaf factors
  c64* G32 = nullptr; // complex64 copy (mixed)
  long long g_total = 0;
  int* d_info = nullptr;
  // outer-loop buffers
  std::vector<DevBuf> scratch;
  c128* d_partial = nullptr;
  size_t partial_cap = 0;
  // live kernel timing (HIP events on the library stream), per kernel family
  bool prof = false;
  struct ProfRec {
    int fam;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<ProfRec> prof_open;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[4] = {0, 0, 0, 0};
  double prof_bytes[4] = {0, 0, 0, 0};
  double prof_flops[4] = {0, 0, 0, 0};
  long long prof_n[4] = {0, 0, 0, 0};
  int* poll = nullptr;          // pinned host words polled by the outer loop
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  std::vector<DevBuf> allocs;
};

namespace {

#define HH_CHECK(expr)                                                   \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess) return device_fail(c, #expr, e_);              \
  } while (0)

#define HH_TRY(expr)                       \
  do {                                     \
    hh_status s_ = (expr);                 \
    if (s_ != HH_OK) return s_;            \
  } while (0)

hh_status device_fail(hh_ctx* c, const char* what, hipError_t e) {
  c->poisoned = true;
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return HH_EDEVICE;
}

hh_status fail(hh_ctx* c, hh_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

template <typename T>
hh_status dalloc(hh_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return HH_OK;
  const size_t bytes = count * sizeof(T);
  void* q = devpool::acquire(bytes, c->stream);
  if (!q) return fail(c, HH_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  c->allocs.push_back(DevBuf{q, bytes});
  *p = reinterpret_cast<T*>(q);
  return HH_OK;
}

// Back to the pool; work already enqueued on the context stream may still use it.
void dfree(hh_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find_if(c->allocs.begin(), c->allocs.end(), [p](const DevBuf& b) { return b.p == p; });
  if (it == c->allocs.end()) return;
  devpool::release(p, it->bytes, c->stream);
  c->allocs.erase(it);
}

template <typename T>
hh_status upload(hh_ctx* c, T** dst, const std::vector<T>& src) {
  if (*dst) {
    dfree(c, *dst);
    *dst = nullptr;
  }
  if (src.empty()) return HH_OK;
  HH_TRY(dalloc(c, dst, src.size()));
  HH_CHECK(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HH_CHECK(hipStreamSynchronize(c->stream));
  return HH_OK;
}

hh_status sync(hh_ctx* c) {
  HH_CHECK(hipStreamSynchronize(c->stream));
  return HH_OK;
}

hh_status push_boxes(hh_ctx* c, Level& L) { return upload(c, &L.d, L.hb); }

// Runs fn(i) for i in [0, n) on up to 8 host threads (on the calling thread
// alone for small n); false when a worker ran out of host memory.
template <typename F>
bool parallel_for(int n, F fn) {
  const long long hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = (int)std::min<long long>({8LL, hw, (n + 63LL) / 64});
  std::atomic<int> next{0};
  std::atomic<bool> ok{true};
  auto work = [&]() {
    try {
      for (int i; ok.load(std::memory_order_relaxed) && (i = next.fetch_add(1)) < n;) fn(i);
    } catch (const std::bad_alloc&) {
      ok = false;
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) {
    try {
      th.emplace_back(work);
    } catch (const std::system_error&) {
      break;  // fewer threads: the calling thread takes what is left
    }
  }
  work();
  for (std::thread& t : th) t.join();
  return ok.load();
}

// Groups the leaves by key(ny) (ascending key, leaves ascending within a group).
template <typename F>
hh_status group_leaves(hh_ctx* c, const Level& L, F key, std::vector<LeafGroup>& groups, int** d_order) {
  std::vector<int> idx(L.nbox);
  for (int i = 0; i < L.nbox; ++i) idx[i] = i;
  // by group, and within a group the largest leaves (longest line chains) first,
  // so that the critical chains start at once and the short ones fill in behind
  auto size = [&](int i) { return (long long)L.hb[i].nx * L.hb[i].ny * L.hb[i].ny; };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    const int ka = key(L.hb[a].ny), kb = key(L.hb[b].ny);
    return ka != kb ? ka < kb : size(a) > size(b);
  });
  groups.clear();
  for (int t = 0; t < L.nbox; ++t) {
    const int k = key(L.hb[idx[t]].ny);
    if (groups.empty() || groups.back().key != k) {
      LeafGroup g;
      g.key = k;
      g.start = t;
      groups.push_back(g);
    }
    groups.back().count += 1;
    groups.back().max_ny = std::max(groups.back().max_ny, L.hb[idx[t]].ny);
  }
  return upload(c, d_order, idx);
}

// Grow the work buffers of levels lo..L to hold q columns.
hh_status ensure_work(hh_ctx* c, int lo, int q) {
  for (int l = lo; l <= c->L; ++l) {
    Level& L = c->lv[l];
    if (L.qcap >= q) continue;
    ++c->epoch;
    for (c128** b : {&L.R, &L.X, &L.T, &L.E, &L.U, &L.cvec, &L.yvec, &L.W, &L.RP}) {
      dfree(c, *b);
      *b = nullptr;
    }
    const size_t n = (size_t)L.total * q;
    HH_TRY(dalloc(c, &L.R, n));
    HH_TRY(dalloc(c, &L.X, n));
    HH_TRY(dalloc(c, &L.T, n));
    HH_TRY(dalloc(c, &L.E, n));
    HH_TRY(dalloc(c, &L.U, n));
    if (L.nc_total > 0) {
      HH_TRY(dalloc(c, &L.cvec, (size_t)L.nc_total * q));
      HH_TRY(dalloc(c, &L.yvec, (size_t)L.nc_total * q));
    }
    if (l == c->L) HH_TRY(dalloc(c, &L.W, (size_t)2 * L.nbox * L.max_ny * q));
    if (l < c->L) {
      const Level& Ch = c->lv[l + 1];
      L.rp_len = restrict_workspace(std::max(Ch.n_rchunks, 1), std::max(Ch.rmax, 1), q);
      HH_TRY(dalloc(c, &L.RP, (size_t)L.rp_len));
    }
    L.qcap = q;
  }
  return HH_OK;
}

hh_status ensure_poll(hh_ctx* c) {
  if (c->poll) return HH_OK;
  void* p = nullptr;
  if (hipHostMalloc(&p, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, HH_ENOMEM, "hipHostMalloc failed");
  }
  c->poll = reinterpret_cast<int*>(p);
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&c->poll_ev[i], hipEventDisableTiming) != hipSuccess)
      return device_fail(c, "hipEventCreateWithFlags", hipGetLastError());
  return HH_OK;
}

hh_status ensure_partial(hh_ctx* c, size_t count) {
  if (c->partial_cap >= count) return HH_OK;
  ++c->epoch;
  dfree(c, c->d_partial);
  c->d_partial = nullptr;
  HH_TRY(dalloc(c, &c->d_partial, count));
  c->partial_cap = count;
  return HH_OK;
}

// ------------------------------------------------------------------ live kernel timing
hipEvent_t prof_event(hh_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  hh_ctx* c;
  int fam;
  double bytes, flops;
  hipEvent_t a = nullptr;
  ProfScope(hh_ctx* c_, int fam_, double bytes_, double flops_) : c(c_), fam(fam_), bytes(bytes_), flops(flops_) {
    if (c->prof && !c->capturing && (a = prof_event(c))) (void)hipEventRecord(a, c->stream);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->prof_open.push_back({fam, a, b, bytes, flops});
  }
};

// fold finished event pairs into the totals (after a stream synchronisation)
void prof_collect(hh_ctx* c) {
  for (auto& r : c->prof_open) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_ms[r.fam] += ms;
      c->prof_bytes[r.fam] += r.bytes;
      c->prof_flops[r.fam] += r.flops;
      c->prof_n[r.fam] += 1;
    }
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof_open.clear();
}

// algorithmic traffic and work of one leaf-solve launch over q columns: every
// G_j streamed once per sweep (2 nx - 1 blocks of b^2), right-hand side read,
// solution written in the forward sweep, read and written in the backward one
void leaf_solve_cost(const Level& L, int q, size_t gbytes, double& bytes, double& flops) {
  bytes = 0.0;
  flops = 0.0;
  for (const BoxDev& b : L.hb) {
    const double bb = (double)b.ny * b.ny;
    bytes += (2.0 * b.nx - 1.0) * bb * gbytes + 4.0 * q * (double)b.n * 16.0;
    flops += 8.0 * (2.0 * b.nx - 1.0) * bb * q;
  }
}

// ------------------------------------------------------------------ the sweeps
hh_status solve_level(hh_ctx* c, int l, int q, const c128* rhs, c128* x);
hh_status leaf_solve(hh_ctx* c, int q, const c128* rhs, c128* x, const BoxDev* par, c128* out);

// out = B_l(r) for every box of level l: smoother over the children, then the
// coarse correction of each box's own coarse space (eqs. (sub1)-(coarse1)).
// Leaf children read R_i r from the parent vector and write P_i x into it
// directly; inner levels go through their own level buffers.
hh_status two_level(hh_ctx* c, int l, int q, const c128* r, c128* out) {
  Level& P = c->lv[l];
  Level& Ch = c->lv[l + 1];
  if (l + 1 == c->L) {
    HH_TRY(leaf_solve(c, q, r, Ch.X, P.d, out));
  } else {
    HH_CHECK(launch_gather_children(Ch.d, Ch.nbox, Ch.max_n, P.d, q, r, Ch.R, c->stream));
    HH_TRY(solve_level(c, l + 1, q, Ch.R, Ch.X));
    HH_CHECK(launch_scatter_owned(Ch.d, Ch.nbox, Ch.max_own, P.d, q, Ch.X, out, c->stream));
  }
  if (P.has_coarse) {
    HH_CHECK(launch_apply_box(c->d_ops, P.d, P.nbox, P.max_n, q, out, r, P.T, 1, c->stream, c->act));
    if (P.rp_len < restrict_workspace(Ch.n_rchunks, Ch.rmax, q))
      return fail(c, HH_EDEVICE, "coarse restriction workspace smaller than the launch needs");
    HH_CHECK(launch_coarse_restrict(Ch.d, Ch.nbox, Ch.d_rchunks, Ch.d_rcbase, Ch.n_rchunks, P.d, P.dp, Ch.rmax, q, Ch.C,
                                    P.T, P.RP, P.cvec, c->act, c->stream));
    HH_CHECK(launch_coarse_gemv(P.dp, P.nbox, P.max_nc, q, P.Ainv, P.cvec, P.yvec, c->stream));
    HH_CHECK(launch_coarse_prolong(Ch.d, Ch.d_pgroups, Ch.n_pgroups, Ch.rmax, P.d, P.dp, q, Ch.C, P.yvec, out,
                                   c->act, c->stream));
  }
  return HH_OK;
}

// Exact solves of every leaf box (the local problems of eq. (sub1)); see
// launch_leaf_solve for the in-place parent mode (par, out).
hh_status leaf_solve(hh_ctx* c, int q, const c128* rhs, c128* x, const BoxDev* par, c128* out) {
  Level& Lv = c->lv[c->L];
  double bytes = 0.0, flops = 0.0;
  if (c->prof) leaf_solve_cost(Lv, q, c->precision == HH_MIXED ? 8 : 16, bytes, flops);
  ProfScope ps(c, 0, bytes, flops);
  if (Lv.qcap < q) return fail(c, HH_EDEVICE, "leaf solve work space smaller than the launch needs");
  auto launch = [&](const LeafGroup& g, int qb) {
    const int* lidx = Lv.d_sweep_order + g.start;
    if (c->precision == HH_MIXED)
      return launch_leaf_solve<float>(c->d_ops, Lv.d, lidx, g.count, g.key, Lv.max_ny, q, qb, c->G32, rhs, x, Lv.W,
                                      par, out, c->act, c->stream);
    return launch_leaf_solve<double>(c->d_ops, Lv.d, lidx, g.count, g.key, Lv.max_ny, q, qb, c->G, rhs, x, Lv.W, par,
                                     out, c->act, c->stream);
  };
  for (LeafGroup& g : Lv.sweep_groups) {
    if (c->autotune && !c->capturing && g.qb_q != q) {
      // the autotuner: time every column-group width on this launch's own data
      // (each computes the same result, so the trial runs are harmless) and keep
      // the fastest for this q
      hipEvent_t e0 = prof_event(c), e1 = prof_event(c);
      if (!e0 || !e1) return device_fail(c, "hipEventCreate", hipErrorOutOfMemory);
      float best = 3.0e38f;
      int bq = 0;
      for (int qb : {1, 2, 4}) {
        if (qb > 1 && qb > q) continue;
        for (int rep = 0; rep < 2; ++rep) {
          HH_CHECK(hipEventRecord(e0, c->stream));
          HH_CHECK(launch(g, qb));
          HH_CHECK(hipEventRecord(e1, c->stream));
          HH_CHECK(hipEventSynchronize(e1));
          float ms = 0.0f;
          HH_CHECK(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best) {
            best = ms;
            bq = qb;
          }
        }
      }
      c->ev_pool.push_back(e0);
      c->ev_pool.push_back(e1);
      g.qb = bq;
      g.qb_q = q;
    }
    HH_CHECK(launch(g, g.qb_q == q ? g.qb : 0));
  }
  return HH_OK;
}

// x = S_l(rhs) for every box of level l >= 1: exact leaf solve, or n_i
// two-level steps from zero on the box problem.
hh_status solve_level(hh_ctx* c, int l, int q, const c128* rhs, c128* x) {
  Level& Lv = c->lv[l];
  if (l == c->L) return leaf_solve(c, q, rhs, x, nullptr, nullptr);
  const int ni = std::max(1, c->inner[l]);
  HH_TRY(two_level(c, l, q, rhs, x));
  for (int it = 1; it < ni; ++it) {
    HH_CHECK(launch_apply_box(c->d_ops, Lv.d, Lv.nbox, Lv.max_n, q, x, rhs, Lv.E, 1, c->stream));
    HH_TRY(two_level(c, l, q, Lv.E, Lv.U));
    HH_CHECK(launch_add_masked(Lv.U, x, (long long)Lv.total * q, 1, nullptr, c->stream));
  }
  return HH_OK;
}

// Entry points start here: a HIP error left in this thread's last-error slot by an
// earlier, unrelated call (the caller's own or a failed allocation handled
// elsewhere) is cleared, so that the checks after this call's launches see only
// their own errors.
hh_status check_usable(hh_ctx* c) {
  if (!c) return HH_EINVAL;
  (void)hipGetLastError();
  if (c->poisoned) return fail(c, HH_EDEVICE, "context poisoned by an earlier device error: " + c->err);
  return HH_OK;
}

// message of this thread's last failed set-up (its context no longer exists)
thread_local std::string t_setup_err;

hh_status check_built(hh_ctx* c) {
  for (int l = 1; l <= c->L; ++l)
    if (!c->lv[l].built) return fail(c, HH_ESTATE, "hh_build_coarse has not run for level " + std::to_string(l));
  return HH_OK;
}

// Outer-loop systems for q right-hand sides: system b = p q + c is column c of
// problem p, the segment of level-0 box p that holds it.
hh_status ensure_segs(hh_ctx* c, int q) {
  if (c->sg_q == q) return HH_OK;
  ++c->epoch;
  const Level& R = c->lv[0];
  const int S = R.nbox * q;
  std::vector<long long> off(S);
  std::vector<int> len(S), nb(S);
  std::vector<int2> ch;
  int nbmax = 0;
  for (int p = 0; p < R.nbox; ++p)
    for (int col = 0; col < q; ++col) {
      const int b = p * q + col;
      off[b] = R.hb[p].voff * q + (long long)col * R.hb[p].n;
      len[b] = R.hb[p].n;
      nb[b] = multidot_nblocks(len[b]);
      nbmax = std::max(nbmax, nb[b]);
      for (int k = 0; k < nb[b]; ++k) ch.push_back(make_int2(b, k));
    }
  c->sg_q = 0;
  HH_TRY(upload(c, &c->d_seg_off, off));
  HH_TRY(upload(c, &c->d_seg_len, len));
  HH_TRY(upload(c, &c->d_seg_nb, nb));
  HH_TRY(upload(c, &c->d_seg_chunk, ch));
  c->sg.off = c->d_seg_off;
  c->sg.len = c->d_seg_len;
  c->sg.nb = c->d_seg_nb;
  c->sg.chunk = c->d_seg_chunk;
  c->sg.S = S;
  c->sg.G = (int)ch.size();
  c->sg.NBmax = nbmax;
  c->sg_q = q;
  return HH_OK;
}

// Device norms of the outer-loop systems (ensure_segs done): out[b] = ||x_b||_2 on the host.
hh_status norms(hh_ctx* c, const c128* x, c128* dtmp, std::vector<double>& out) {
  const int S = c->sg.S;
  HH_TRY(ensure_partial(c, (size_t)S * c->sg.NBmax));
  HH_CHECK(launch_multidot(1, c->sg, x, 0, x, c->d_partial, dtmp, c->stream));
  std::vector<c128> h(S);
  HH_CHECK(hipMemcpyAsync(h.data(), dtmp, S * sizeof(c128), hipMemcpyDeviceToHost, c->stream));
  HH_TRY(sync(c));
  out.resize(S);
  for (int b = 0; b < S; ++b) out[b] = std::sqrt(std::max(h[b].x, 0.0));
  return HH_OK;
}

}  // namespace

extern "C" {

const char* hh_status_string(hh_status s) {
  switch (s) {
    case HH_OK: return "HH_OK";
    case HH_EINVAL: return "HH_EINVAL";
    case HH_ENOMEM: return "HH_ENOMEM";
    case HH_EDEVICE: return "HH_EDEVICE";
    case HH_ENOTCONV: return "HH_ENOTCONV";
    case HH_ESINGULAR: return "HH_ESINGULAR";
    case HH_ESTATE: return "HH_ESTATE";
    case HH_EUNSUPPORTED: return "HH_EUNSUPPORTED";
  }
  return "unknown";
}

const char* hh_last_error(const hh_ctx* c) {
  if (c) return c->err.c_str();
  return t_setup_err.empty() ? "null context" : t_setup_err.c_str();
}

hh_status hh_destroy(hh_ctx* c) {
  if (!c) return HH_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipGraphExec_t e : c->gw.exec)
    if (e) (void)hipGraphExecDestroy(e);
  for (int i = 0; i < 2; ++i)
    if (c->poll_ev[i]) (void)hipEventDestroy(c->poll_ev[i]);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& r : c->prof_open) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (c->poll) (void)hipHostFree(c->poll);
  // the stream was synchronised above: the blocks go back idle, and blocks this
  // context released earlier stop referring to the stream (the caller may
  // destroy it once its contexts are gone)
  for (const DevBuf& b : c->allocs) devpool::release(b.p, b.bytes, c->stream, true);
  c->allocs.clear();
  devpool::forget_stream(c->stream);
  delete c;
  (void)hipGetLastError();  // clean-up ignores errors; leave none behind for the caller's next call
  return HH_OK;
}

hh_status hh_release_cached_memory(int64_t* bytes) {
  const size_t n = devpool::trim();
  if (bytes) *bytes = (int64_t)n;
  return HH_OK;
}

hh_status hh_setup(const hh_operator* A, const hh_decomposition* d, const hh_options* o, hh_ctx** out) {
  return hh_setup_batch(1, A, d, o, out);
}

hh_status hh_setup_batch(int32_t nprob, const hh_operator* A, const hh_decomposition* d, const hh_options* o,
                         hh_ctx** out) {
  t_setup_err.clear();
  (void)hipGetLastError();
  if (!A || !d || !out || nprob < 1) return HH_EINVAL;
  *out = nullptr;
  std::vector<Geometry> parts(nprob);
  for (int p = 0; p < nprob; ++p) {
    const hh_operator& Ap = A[p];
    if (Ap.dim != 1 && Ap.dim != 2) return HH_EINVAL;
    if (Ap.n_cells < 2 || Ap.n_cells > (1 << 15)) return HH_EINVAL;
    if (Ap.dim != A[0].dim || d[p].levels != d[0].levels) return HH_EINVAL;
    const long long N1 = Ap.n_cells + 1;
    const long long nn = Ap.dim == 2 ? N1 * N1 : N1;
    if (Ap.k) {
      for (long long i = 0; i < nn; ++i)
        if (!std::isfinite(Ap.k[i]) || Ap.k[i] < 0.0) return HH_EINVAL;
    } else if (!std::isfinite(Ap.k_const) || Ap.k_const < 0.0) {
      return HH_EINVAL;
    }
    if (!build_geometry(Ap.dim, Ap.n_cells, d[p].levels, d[p].m, d[p].overlap_cells, parts[p]).empty())
      return HH_EINVAL;
  }
  hh_ctx* c = new (std::nothrow) hh_ctx();
  if (!c) return HH_ENOMEM;
  if (o) {
    c->stream = reinterpret_cast<hipStream_t>(o->stream);
    c->precision = o->precision == HH_MIXED ? HH_MIXED : HH_FP64;
    c->outer = o->outer == HH_STATIONARY ? HH_STATIONARY : HH_GMRES;
    c->restart = o->gmres_restart > 0 ? std::min(o->gmres_restart, 120) : 50;
    c->reorth_eta = o->full_reorth ? 2.0 : 0.125;
    c->autotune = o->autotune != 0;
    c->graphs = o->graphs != 0;
  }
  if (!merge_geometries(parts, c->geo).empty()) {
    delete c;
    return HH_EINVAL;
  }
  parts.clear();
  c->nprob = nprob;
  c->L = d->levels;
  // inner steps per level: the largest any problem asks for (the batch advances together)
  c->inner.assign(c->L + 1, 1);
  for (int p = 0; p < nprob; ++p)
    for (int l = 1; l <= c->L; ++l) c->inner[l] = std::max(c->inner[l], std::max(1, (int)d[p].inner_iters[l - 1]));
  hh_status st = HH_OK;
  auto bail = [&](hh_status s) {
    t_setup_err = c->err;
    hh_destroy(c);
    return s;
  };
  // operators: one table row per problem, wavenumbers concatenated
  std::vector<double> kv;
  std::vector<long long> koff(nprob, -1);
  for (int p = 0; p < nprob; ++p) {
    const hh_operator& Ap = A[p];
    const long long N1 = Ap.n_cells + 1;
    const long long nn = Ap.dim == 2 ? N1 * N1 : N1;
    if (Ap.k) {
      koff[p] = (long long)kv.size();
      kv.insert(kv.end(), Ap.k, Ap.k + nn);
    }
  }
  if ((st = upload(c, &c->d_k, kv)) != HH_OK) return bail(st);
  c->hops.resize(nprob);
  for (int p = 0; p < nprob; ++p) {
    OpDev& op = c->hops[p];
    op.kc = A[p].k_const;
    op.h = 1.0 / A[p].n_cells;
    op.ih2 = (double)A[p].n_cells * (double)A[p].n_cells;
    op.N1 = A[p].n_cells + 1;
    op.dim = A[p].dim;
    op.k = koff[p] >= 0 ? c->d_k + koff[p] : nullptr;
  }
  if ((st = upload(c, &c->d_ops, c->hops)) != HH_OK) return bail(st);
  // levels
  c->lv.resize(c->L + 1);
  for (int l = 0; l <= c->L; ++l) {
    Level& Lv = c->lv[l];
    const std::vector<HBox>& gb = c->geo.levels[l];
    Lv.nbox = (int)gb.size();
    Lv.hb.resize(Lv.nbox);
    std::vector<int> ifidx;
    long long off = 0;
    for (int i = 0; i < Lv.nbox; ++i) {
      const HBox& h = gb[i];
      BoxDev& b = Lv.hb[i];
      std::memset(&b, 0, sizeof(b));
      b.p0 = h.p0; b.p1 = h.p1; b.q0 = h.q0; b.q1 = h.q1;
      b.op0 = h.op0; b.op1 = h.op1; b.oq0 = h.oq0; b.oq1 = h.oq1;
      b.nx = h.nx(); b.ny = h.ny(); b.n = h.n();
      b.parent = h.parent < 0 ? 0 : h.parent;
      b.prob = h.prob;
      if (l > 0) {
        const HBox& ph = c->geo.levels[l - 1][h.parent];
        b.pp0 = ph.p0; b.pq0 = ph.q0; b.pny = ph.ny();
      }
      b.m_in = (int)h.iface.size();
      b.if_off = (int)ifidx.size();
      ifidx.insert(ifidx.end(), h.iface.begin(), h.iface.end());
      b.n_own = h.n_own();
      b.own_ny = h.oq1 - h.oq0 + 1;
      b.voff = off;
      off += b.n;
      Lv.max_n = std::max(Lv.max_n, b.n);
      Lv.max_nx = std::max(Lv.max_nx, b.nx);
      Lv.max_ny = std::max(Lv.max_ny, b.ny);
      Lv.max_own = std::max(Lv.max_own, b.n_own);
    }
    Lv.total = off;
    if ((st = upload(c, &Lv.d_if, ifidx)) != HH_OK) return bail(st);
  }
  // leaf factor storage
  Level& leaf = c->lv[c->L];
  if (leaf.max_ny > 256) {
    c->err = "leaf boxes wider than 256 nodes along q are not supported";
    return bail(HH_EUNSUPPORTED);
  }
  long long goff = 0;
  for (BoxDev& b : leaf.hb) {
    b.goff = goff;
    goff += (long long)b.nx * b.ny * b.ny;
  }
  c->g_total = goff;
  for (int l = 0; l <= c->L; ++l)
    if ((st = push_boxes(c, c->lv[l])) != HH_OK) return bail(st);
  if ((st = group_leaves(c, leaf, leaf_sweep_bucket, leaf.sweep_groups, &leaf.d_sweep_order)) != HH_OK ||
      (st = group_leaves(c, leaf, leaf_factor_bucket, leaf.factor_groups, &leaf.d_factor_order)) != HH_OK)
    return bail(st);
  // tail padding (zeroed): the sweeps read whole column slices and row groups past a line's end
  const long long gpad = 256LL * 256LL;
  if ((st = dalloc(c, &c->G, (size_t)(goff + gpad))) != HH_OK) return bail(st);
  if (launch_fill_zero(c->G + goff, gpad * (long long)sizeof(c128), c->stream) != hipSuccess)
    return bail(device_fail(c, "fill", hipGetLastError()));
  const int ninfo = 3 * leaf.nbox;
  if ((st = dalloc(c, &c->d_info, (size_t)std::max(ninfo, 4096))) != HH_OK) return bail(st);
  for (const LeafGroup& g : leaf.factor_groups)
    if (launch_leaf_factor(c->d_ops, leaf.d, leaf.nbox, leaf.d_factor_order + g.start, g.count, g.max_ny, c->G,
                           c->d_info, c->stream) != hipSuccess)
      return bail(device_fail(c, "leaf factor", hipGetLastError()));
  std::vector<int> info(ninfo);
  if (hipMemcpyAsync(info.data(), c->d_info, ninfo * sizeof(int), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(device_fail(c, "leaf factor sync", hipGetLastError()));
  for (int i = 0; i < ninfo; ++i)
    if (info[i] != 0) {
      const int lf = i < 2 * leaf.nbox ? i / 2 : i - 2 * leaf.nbox;
      c->err = "zero pivot in the factorisation of leaf " + std::to_string(lf);
      return bail(HH_ESINGULAR);
    }
  if (c->precision == HH_MIXED) {
    if ((st = dalloc(c, &c->G32, (size_t)(goff + gpad))) != HH_OK) return bail(st);
    if (launch_fill_zero(c->G32 + goff, gpad * (long long)sizeof(c64), c->stream) != hipSuccess)
      return bail(device_fail(c, "fill", hipGetLastError()));
    if (launch_f64_to_f32(c->G, c->G32, goff, c->stream) != hipSuccess)
      return bail(device_fail(c, "convert", hipGetLastError()));
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(device_fail(c, "sync", hipGetLastError()));
    dfree(c, c->G);
    c->G = nullptr;
  }
  *out = c;
  return HH_OK;
}

hh_status hh_level_info(const hh_ctx* cc, int32_t level, int32_t rank, int32_t oversample, int32_t* n_boxes,
                        int32_t* m_in, int32_t* r, int32_t* s) {
  if (!cc) return HH_EINVAL;
  if (level < 0 || level > cc->L || rank < 0 || oversample < 0) return HH_EINVAL;
  const std::vector<HBox>& gb = cc->geo.levels[level];
  if (n_boxes) *n_boxes = (int32_t)gb.size();
  for (size_t i = 0; i < gb.size(); ++i) {
    const int mi = (int)gb[i].iface.size();
    const long long rr = std::min<long long>((long long)rank * gb[i].n_if, mi);
    const long long ss = rr > 0 ? std::min<long long>(rr + oversample, mi) : 0;
    if (m_in) m_in[i] = mi;
    if (r) r[i] = (int32_t)rr;
    if (s) s[i] = (int32_t)ss;
  }
  return HH_OK;
}

hh_status hh_problem_layout(const hh_ctx* c, int32_t* nprob, int64_t* n_nodes, int64_t* offset) {
  if (!c) return HH_EINVAL;
  const Level& R = c->lv[0];
  if (nprob) *nprob = R.nbox;
  for (int p = 0; p < R.nbox; ++p) {
    if (n_nodes) n_nodes[p] = R.hb[p].n;
    if (offset) offset[p] = R.hb[p].voff;
  }
  return HH_OK;
}

hh_status hh_sweep_plan(const hh_ctx* c, int32_t* ngroups, int32_t* bucket, int32_t* count, int32_t* max_width,
                        int32_t* qb, int32_t* tuned_for) {
  if (!c) return HH_EINVAL;
  const Level& Lv = c->lv[c->L];
  if (ngroups) *ngroups = (int32_t)Lv.sweep_groups.size();
  for (size_t i = 0; i < Lv.sweep_groups.size(); ++i) {
    const LeafGroup& g = Lv.sweep_groups[i];
    if (bucket) bucket[i] = g.key;
    if (count) count[i] = g.count;
    if (max_width) max_width[i] = g.max_ny;
    if (qb) qb[i] = g.qb;
    if (tuned_for) tuned_for[i] = g.qb_q;
  }
  return HH_OK;
}

hh_status hh_build_coarse(hh_ctx* c, int32_t level, int32_t rank, int32_t oversample, const void* omega) {
  HH_TRY(check_usable(c));
  if (level < 1 || level > c->L || rank < 0 || oversample < 0)
    return fail(c, HH_EINVAL, "level must be in 1..levels; rank and oversample non-negative");
  if (level < c->L && !c->lv[level + 1].built)
    return fail(c, HH_ESTATE, "build the coarse spaces from the finest level up");
  Level& Lv = c->lv[level];
  Level& P = c->lv[level - 1];
  const std::vector<HBox>& gb = c->geo.levels[level];
  const std::vector<HBox>& pgb = c->geo.levels[level - 1];
  // ranks and sketch widths
  int rmax = 0, smax = 0;
  for (int i = 0; i < Lv.nbox; ++i) {
    const int mi = (int)gb[i].iface.size();
    const int rr = (int)std::min<long long>((long long)rank * gb[i].n_if, mi);
    const int ss = rr > 0 ? (int)std::min<long long>((long long)rr + oversample, mi) : 0;
    Lv.hb[i].r = rr;
    Lv.hb[i].s = ss;
    rmax = std::max(rmax, rr);
    smax = std::max(smax, ss);
  }
  if (smax > 128) return fail(c, HH_EUNSUPPORTED, "sketch width above 128 is not supported");
  if (rmax > 0 && !omega) return fail(c, HH_EINVAL, "omega is required when the rank is positive");
  // invalidate every coarser level: their sub-solves change with this one
  for (int l = 1; l < level; ++l) c->lv[l].built = false;
  ++c->epoch;
  Lv.rank = rank;
  Lv.rmax = rmax;
  Lv.smax = smax;
  // parents' coarse layout
  P.hp.assign(P.nbox, ParentDev{});
  long long nc_tot = 0, nc2 = 0;
  int max_nc = 0;
  for (int p = 0; p < P.nbox; ++p) {
    ParentDev& pd = P.hp[p];
    const HBox& ph = pgb[p];
    int nc = 0;
    pd.child0 = ph.children.empty() ? 0 : ph.children.front();
    pd.nchild = (int)ph.children.size();
    for (int ch : ph.children) {
      Lv.hb[ch].cidx = nc;
      nc += Lv.hb[ch].r;
    }
    pd.n_c = nc;
    pd.aoff = nc2;
    pd.yoff = nc_tot;
    nc2 += (long long)nc * nc;
    nc_tot += nc;
    max_nc = std::max(max_nc, nc);
  }
  for (c128** b : {&P.Ainv, &P.Araw, &P.cvec, &P.yvec}) {
    dfree(c, *b);
    *b = nullptr;
  }
  dfree(c, P.d_piv);
  P.d_piv = nullptr;
  dfree(c, Lv.C);
  Lv.C = nullptr;
  dfree(c, Lv.AC);
  Lv.AC = nullptr;
  P.nc_total = nc_tot;
  P.nc2_total = nc2;
  P.max_nc = max_nc;
  P.has_coarse = false;
  P.qcap = 0;  // forces cvec/yvec reallocation with the new size
  Lv.sigma.assign((size_t)Lv.nbox * std::max(smax, 1), 0.0);
  if (rmax == 0) {
    HH_TRY(push_boxes(c, Lv));
    HH_TRY(upload(c, &P.dp, P.hp));
    Lv.built = true;
    return HH_OK;
  }
  // trace tables (geometry only; cached).  Every box's tables are independent:
  // they are built on host threads, then packed at offsets from a prefix sum.
  if (!Lv.tables) {
    std::vector<std::vector<TraceRow>> trows(Lv.nbox);
    std::vector<std::vector<AdjEntry>> tadj(Lv.nbox);
    std::vector<int> nseg(Lv.nbox, 0);
    if (!parallel_for(Lv.nbox, [&](int i) {
          trace_tables(c->geo, level, i, trows[i], tadj[i]);
          int k = 0, prev = -1;
          for (const AdjEntry& e : tadj[i])
            if (e.yl != prev) {
              ++k;
              prev = e.yl;
            }
          nseg[i] = k;
        }))
      return fail(c, HH_ENOMEM, "out of host memory for the interface-map tables");
    long long nr = 0, ns = 0, na = 0;
    std::vector<long long> aoff(Lv.nbox);
    for (int i = 0; i < Lv.nbox; ++i) {
      BoxDev& b = Lv.hb[i];
      b.tr_off = (int)nr;
      b.tr_cnt = (int)trows[i].size();
      b.adj_off = (int)ns;
      b.adj_cnt = nseg[i];
      Lv.max_tr = std::max(Lv.max_tr, b.tr_cnt);
      aoff[i] = na;
      nr += b.tr_cnt;
      ns += nseg[i];
      na += (long long)tadj[i].size();
    }
    if (na >= (1LL << 31) || nr >= (1LL << 31)) return fail(c, HH_EUNSUPPORTED, "interface-map tables too large");
    std::vector<int2> rows(nr);
    std::vector<int> seg_ptr(ns + 1), seg_y(ns);
    std::vector<int4> adj(na);
    parallel_for(Lv.nbox, [&](int i) {
      const BoxDev& b = Lv.hb[i];
      for (int t = 0; t < b.tr_cnt; ++t) rows[b.tr_off + t] = make_int2(trows[i][t].j, trows[i][t].xl);
      long long a = aoff[i];
      int sg = b.adj_off, prev = -1;
      for (const AdjEntry& e : tadj[i]) {
        if (e.yl != prev) {
          seg_ptr[sg] = (int)a;
          seg_y[sg] = e.yl;
          ++sg;
          prev = e.yl;
        }
        adj[a++] = make_int4(e.row, e.dp, e.dq, 0);
      }
    });
    seg_ptr[ns] = (int)na;
    HH_TRY(upload(c, &Lv.d_rows, rows));
    HH_TRY(upload(c, &Lv.d_seg_ptr, seg_ptr));
    HH_TRY(upload(c, &Lv.d_seg_y, seg_y));
    HH_TRY(upload(c, &Lv.d_adj, adj));
    Lv.tables = true;
  }
  // coarse block storage, dilated owned boxes, Galerkin pairs
  long long coff = 0, acoff = 0;
  std::vector<int4> dil(Lv.nbox);
  int max_dil = 0;
  for (int i = 0; i < Lv.nbox; ++i) {
    BoxDev& b = Lv.hb[i];
    const HBox& h = gb[i];
    const HBox& ph = pgb[h.parent];
    b.coff = coff;
    coff += (long long)b.r * b.n_own;
    int4 d4;
    d4.x = std::max(h.op0 - 1, ph.p0);
    d4.y = std::min(h.op1 + 1, ph.p1);
    d4.z = c->geo.dim == 2 ? std::max(h.oq0 - 1, ph.q0) : 0;
    d4.w = c->geo.dim == 2 ? std::min(h.oq1 + 1, ph.q1) : 0;
    dil[i] = d4;
    const int nd = (d4.y - d4.x + 1) * (d4.w - d4.z + 1);
    max_dil = std::max(max_dil, nd);
    b.acoff = acoff;
    acoff += (long long)b.r * nd;
  }
  std::vector<int4> pairs;
  for (int p = 0; p < P.nbox; ++p)
    for (int i : pgb[p].children)
      for (int j : pgb[p].children) {
        const HBox& hi = gb[i];
        const int4& dj = dil[j];
        if (hi.op0 <= dj.y && dj.x <= hi.op1 && hi.oq0 <= dj.w && dj.z <= hi.oq1 && Lv.hb[i].r > 0 &&
            Lv.hb[j].r > 0)
          pairs.push_back(make_int4(i, j, p, 0));
      }
  Lv.max_dil = max_dil;
  Lv.npairs = (int)pairs.size();
  {
    std::vector<int2> rch, pgr;
    std::vector<int> cbase(Lv.nbox, 0);
    const int RC = restrict_chunk_nodes(), PG = prolong_group_nodes();
    for (int i = 0; i < Lv.nbox; ++i) {
      const BoxDev& b = Lv.hb[i];
      cbase[i] = (int)rch.size();
      if (b.r == 0) continue;
      for (int k = 0; k * RC < b.n_own; ++k) rch.push_back(make_int2(i, k));
      for (int k = 0; k * PG < b.n_own; ++k) pgr.push_back(make_int2(i, k));
    }
    Lv.n_rchunks = (int)rch.size();
    Lv.n_pgroups = (int)pgr.size();
    HH_TRY(upload(c, &Lv.d_rchunks, rch));
    HH_TRY(upload(c, &Lv.d_rcbase, cbase));
    HH_TRY(upload(c, &Lv.d_pgroups, pgr));
  }
  HH_TRY(upload(c, &Lv.d_dil, dil));
  HH_TRY(upload(c, &Lv.d_pairs, pairs));
  HH_TRY(push_boxes(c, Lv));
  HH_TRY(upload(c, &P.dp, P.hp));
  HH_TRY(dalloc(c, &Lv.C, (size_t)coff));
  HH_TRY(dalloc(c, &Lv.AC, (size_t)acoff));
  HH_TRY(dalloc(c, &P.Ainv, (size_t)nc2));
  HH_TRY(dalloc(c, &P.Araw, (size_t)nc2));
  HH_TRY(dalloc(c, &P.d_piv, (size_t)P.nbox * max_nc));
  // ---------------------------------------------------------------- sketch Y = T_i Omega_i
  // the sketches run smax columns through this level's boxes and the levels below
  HH_TRY(ensure_work(c, level, std::max(smax, 1)));
  // per-box small-matrix layouts
  std::vector<int> qm(Lv.nbox), qn(Lv.nbox), bm(Lv.nbox), rr(Lv.nbox);
  std::vector<long long> yoff(Lv.nbox), soff(Lv.nbox), bhoff(Lv.nbox), voff(Lv.nbox), omoff(Lv.nbox),
      sgoff(Lv.nbox);
  long long yt = 0, bht = 0, vt = 0, omt = 0;
  int max_mr = 0;
  for (int i = 0; i < Lv.nbox; ++i) {
    const BoxDev& b = Lv.hb[i];
    qm[i] = b.tr_cnt;
    qn[i] = b.s;
    bm[i] = b.m_in;
    rr[i] = b.r;
    yoff[i] = yt;
    yt += (long long)b.tr_cnt * b.s;
    soff[i] = (long long)i * smax * smax;
    sgoff[i] = (long long)i * smax;
    bhoff[i] = bht;
    bht += (long long)b.m_in * b.s;
    voff[i] = vt;
    vt += (long long)b.m_in * b.r;
    omoff[i] = omt;
    omt += (long long)b.m_in * b.s;
    max_mr = std::max(max_mr, b.m_in * std::max(b.r, 1));
  }
  int *d_qm = nullptr, *d_qn = nullptr, *d_bm = nullptr, *d_rr = nullptr;
  long long *d_yoff = nullptr, *d_soff = nullptr, *d_bhoff = nullptr, *d_voff = nullptr, *d_omoff = nullptr,
            *d_sgoff = nullptr;
  c128 *Y = nullptr, *Wk = nullptr, *Rs = nullptr, *Us = nullptr, *BH = nullptr, *V = nullptr;
  double* d_sig = nullptr;
  int* d_drop = nullptr;
  auto cleanup = [&]() {
    for (void* p : std::initializer_list<void*>{d_qm, d_qn, d_bm, d_rr, d_yoff, d_soff, d_bhoff, d_voff, d_omoff,
                                                d_sgoff, Y, Wk, Rs, Us, BH, V, d_sig, d_drop})
      dfree(c, p);
  };
  hh_status st = HH_OK;
  do {
    if ((st = upload(c, &d_qm, qm)) != HH_OK) break;
    if ((st = upload(c, &d_qn, qn)) != HH_OK) break;
    if ((st = upload(c, &d_bm, bm)) != HH_OK) break;
    if ((st = upload(c, &d_rr, rr)) != HH_OK) break;
    if ((st = upload(c, &d_yoff, yoff)) != HH_OK) break;
    if ((st = upload(c, &d_soff, soff)) != HH_OK) break;
    if ((st = upload(c, &d_sgoff, sgoff)) != HH_OK) break;
    if ((st = upload(c, &d_bhoff, bhoff)) != HH_OK) break;
    if ((st = upload(c, &d_voff, voff)) != HH_OK) break;
    if ((st = upload(c, &d_omoff, omoff)) != HH_OK) break;
    const size_t ysz = std::max<long long>(std::max<long long>(yt, bht), (long long)P.nbox * max_nc);
    if ((st = dalloc(c, &Y, ysz)) != HH_OK) break;
    if ((st = dalloc(c, &Wk, ysz)) != HH_OK) break;
    if ((st = dalloc(c, &Rs, (size_t)Lv.nbox * smax * smax)) != HH_OK) break;
    if ((st = dalloc(c, &Us, (size_t)Lv.nbox * smax * smax)) != HH_OK) break;
    if ((st = dalloc(c, &BH, (size_t)std::max<long long>(bht, 1))) != HH_OK) break;
    if ((st = dalloc(c, &V, (size_t)std::max<long long>(vt, 1))) != HH_OK) break;
    if ((st = dalloc(c, &d_sig, (size_t)Lv.nbox * smax)) != HH_OK) break;
    if ((st = dalloc(c, &d_drop, (size_t)Lv.nbox * rmax)) != HH_OK) break;
  } while (false);
  if (st != HH_OK) {
    cleanup();
    return st;
  }
  const c128* Om = reinterpret_cast<const c128*>(omega);
  hipStream_t s = c->stream;
  const int q = smax;
  const long long nlev = Lv.total * q;
#define BC(expr)                                    \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) {                         \
      cleanup();                                    \
      return device_fail(c, #expr, e_);             \
    }                                               \
  } while (0)
#define BT(expr)              \
  do {                        \
    hh_status s2_ = (expr);   \
    if (s2_ != HH_OK) {       \
      cleanup();              \
      return s2_;             \
    }                         \
  } while (0)
  // X = S_i(B_i^T Omega_i)
  BC(launch_fill_zero(Lv.R, nlev * sizeof(c128), s));
  BC(launch_iface_scatter(Lv.d, Lv.nbox, q, Lv.d_if, d_omoff, Om, 0, Lv.R, s));
  BT(solve_level(c, level, q, Lv.R, Lv.X));
  // Y = stacked traces on the neighbours; Q = qr(Y)
  BC(launch_trace(c->d_ops, Lv.d, Lv.nbox, q, Lv.d_rows, d_yoff, Lv.X, Y, s));
  BC(launch_qr(Lv.nbox, d_qm, d_qn, d_yoff, Y, d_soff, Rs, Wk, s));
  // B^H = B_i conj(S_i(conj((B_i^o)^H Q)))
  BC(launch_fill_zero(Lv.R, nlev * sizeof(c128), s));
  BC(launch_trace_adjoint(c->d_ops, Lv.d, Lv.nbox, q, Lv.d_rows, Lv.d_seg_ptr, Lv.d_seg_y, Lv.d_adj, d_yoff, Y, Lv.R,
                          s));
  // (the trace is written conjugated and the gather conjugates what it reads)
  BT(solve_level(c, level, q, Lv.R, Lv.X));
  BC(launch_iface_gather(Lv.d, Lv.nbox, q, Lv.d_if, d_bhoff, Lv.X, BH, 0, 1, s));
  // SVD of B: B^H = Q_B R, R = U_R S V_R^H, V_i = Q_B U_R[:, :r]
  BC(launch_qr(Lv.nbox, d_bm, d_qn, d_bhoff, BH, d_soff, Rs, Wk, s));
  BC(launch_jacobi_svd(Lv.nbox, d_qn, smax, d_soff, Rs, d_soff, Us, d_sig, d_sgoff, s));
  BC(launch_small_gemm(Lv.nbox, max_mr, d_bm, d_qn, d_rr, d_bhoff, BH, d_soff, Us, d_voff, V, s));
  // C_i = P_i S_i(B_i^T V_i)
  BC(launch_fill_zero(Lv.R, (long long)Lv.total * rmax * sizeof(c128), s));
  BC(launch_iface_scatter(Lv.d, Lv.nbox, rmax, Lv.d_if, d_voff, V, 1, Lv.R, s));
  BT(solve_level(c, level, rmax, Lv.R, Lv.X));
  BC(launch_extract_owned(Lv.d, Lv.nbox, Lv.max_own, rmax, Lv.X, Lv.C, s));
  // modes whose extension is (numerically) zero on the owned nodes are dropped
  BC(launch_drop_negligible(Lv.d, Lv.nbox, rmax, kNegligibleMode, Lv.C, d_drop, s));
  // A_c = C^H A_P C, then its inverse
  BC(launch_galerkin_ac(c->d_ops, Lv.d, Lv.nbox, P.d, Lv.d_dil, max_dil, rmax, Lv.C, Lv.AC, s));
  BC(launch_fill_zero(P.Ainv, nc2 * sizeof(c128), s));
  BC(launch_galerkin_blocks(Lv.d, P.dp, Lv.d_pairs, Lv.npairs, rmax, Lv.d_dil, Lv.C, Lv.AC, P.Ainv, s));
  BC(launch_unit_dropped(Lv.d, P.dp, Lv.nbox, rmax, d_drop, P.Ainv, s));
  BC(launch_copy(P.Ainv, P.Araw, nc2, s));
  BC(launch_gj_inverse(P.dp, P.nbox, max_nc, P.Ainv, P.d_piv, Wk, c->d_info, s));
  std::vector<int> info(P.nbox);
  BC(hipMemcpyAsync(info.data(), c->d_info, P.nbox * sizeof(int), hipMemcpyDeviceToHost, s));
  BC(hipMemcpyAsync(Lv.sigma.data(), d_sig, (size_t)Lv.nbox * smax * sizeof(double), hipMemcpyDeviceToHost, s));
  BC(hipStreamSynchronize(s));
  cleanup();
#undef BC
#undef BT
  for (int p = 0; p < P.nbox; ++p)
    if (info[p] != 0) return fail(c, HH_ESINGULAR, "singular coarse matrix A_c of parent " + std::to_string(p));
  P.has_coarse = nc_tot > 0;
  Lv.built = true;
  return HH_OK;
}

hh_status hh_apply_operator(hh_ctx* c, int32_t nrhs, const void* x, const void* b, void* y, int32_t mode) {
  HH_TRY(check_usable(c));
  if (nrhs <= 0 || !x || !y || (mode == 1 && !b) || (mode != 0 && mode != 1)) return fail(c, HH_EINVAL, "bad args");
  Level& R = c->lv[0];
  HH_CHECK(launch_apply_box(c->d_ops, R.d, R.nbox, R.max_n, nrhs, reinterpret_cast<const c128*>(x),
                            reinterpret_cast<const c128*>(b), reinterpret_cast<c128*>(y), mode, c->stream));
  return sync(c);
}

hh_status hh_precondition(hh_ctx* c, int32_t nrhs, const void* r, void* z) {
  HH_TRY(check_usable(c));
  if (nrhs <= 0 || !r || !z) return fail(c, HH_EINVAL, "bad args");
  HH_TRY(check_built(c));
  HH_TRY(ensure_work(c, 0, nrhs));
  HH_TRY(two_level(c, 0, nrhs, reinterpret_cast<const c128*>(r), reinterpret_cast<c128*>(z)));
  return sync(c);
}

}  // extern "C"

namespace {

void drop_graphs(hh_ctx* c) {
  bool any = false;
  for (hipGraphExec_t e : c->gw.exec) any = any || e != nullptr;
  if (any) (void)hipStreamSynchronize(c->stream);  // no replay still in flight
  for (hipGraphExec_t& e : c->gw.exec)
    if (e) (void)hipGraphExecDestroy(e);
  c->gw.exec.clear();
}

// The persistent GMRES work space for q right-hand sides and restart m (the
// captured Arnoldi steps refer to these buffers).
hh_status ensure_gmres(hh_ctx* c, int q, int m) {
  hh_ctx::Gmres& w = c->gw;
  if (w.q == q && w.m == m) return HH_OK;
  drop_graphs(c);
  for (void* p : std::initializer_list<void*>{w.Vb, w.Zb, w.W, w.H, w.cs, w.sn, w.g, w.h1, w.h2, w.tmp, w.y, w.hn,
                                              w.est, w.thr, w.state, w.any, w.need})
    dfree(c, p);
  w = hh_ctx::Gmres();
  ++c->epoch;
  const long long n = c->lv[0].total;
  const int S = c->sg.S;
  HH_TRY(dalloc(c, &w.Vb, (size_t)(m + 1) * q * n));
  HH_TRY(dalloc(c, &w.Zb, (size_t)m * q * n));
  HH_TRY(dalloc(c, &w.W, (size_t)q * n));
  HH_TRY(dalloc(c, &w.H, (size_t)S * (m + 1) * m));
  HH_TRY(dalloc(c, &w.cs, (size_t)S * m));
  HH_TRY(dalloc(c, &w.sn, (size_t)S * m));
  HH_TRY(dalloc(c, &w.g, (size_t)S * (m + 1)));
  HH_TRY(dalloc(c, &w.h1, (size_t)S * (m + 2)));
  HH_TRY(dalloc(c, &w.need, (size_t)S));
  HH_TRY(dalloc(c, &w.h2, (size_t)S * (m + 1)));
  HH_TRY(dalloc(c, &w.tmp, (size_t)S * (m + 1)));
  HH_TRY(dalloc(c, &w.y, (size_t)S * m));
  HH_TRY(dalloc(c, &w.hn, (size_t)S));
  HH_TRY(dalloc(c, &w.est, (size_t)S));
  HH_TRY(dalloc(c, &w.thr, (size_t)S));
  HH_TRY(dalloc(c, &w.state, (size_t)3 * S));
  HH_TRY(dalloc(c, &w.any, (size_t)2));
  w.q = q;
  w.m = m;
  return HH_OK;
}

void release_gmres(hh_ctx* c) {
  hh_ctx::Gmres& w = c->gw;
  drop_graphs(c);
  for (void* p : std::initializer_list<void*>{w.Vb, w.Zb, w.W, w.H, w.cs, w.sn, w.g, w.h1, w.h2, w.tmp, w.y, w.hn,
                                              w.est, w.thr, w.state, w.any, w.need})
    dfree(c, p);
  w = hh_ctx::Gmres();
  ++c->epoch;
}

// One Arnoldi step j for every system: z_j = B v_j, w = A z_j, Gram-Schmidt
// (a second pass where the first cancelled more than reorth_eta), v_{j+1}, and
// the Givens update of the Hessenberg column with the stopping test.  Device
// work only (no allocation, no host synchronisation), so it can be captured.
hh_status arnoldi_step(hh_ctx* c, int q, int j, int maxit) {
  hh_ctx::Gmres& w = c->gw;
  const SegDev& sg = c->sg;
  const int S = sg.S, m = w.m;
  const long long n = c->lv[0].total, vs = (long long)q * n;
  hipStream_t s = c->stream;
  const c128* vj = w.Vb + j * vs;
  c128* zj = w.Zb + j * vs;
  HH_TRY(two_level(c, 0, q, vj, zj));
  const double vbytes = 16.0 * (double)n * q;
  {
    ProfScope ps(c, 3, 2.0 * vbytes, 40.0 * n * q);
    HH_CHECK(launch_apply_box(c->d_ops, c->lv[0].d, c->lv[0].nbox, c->lv[0].max_n, q, zj, nullptr, w.W, 0, s,
                              w.state));
  }
  {
    ProfScope ps(c, 2, vbytes * (j + 1 + (j + 8) / 8), 8.0 * n * q * (j + 1));
    HH_CHECK(launch_multidot(j + 1, sg, w.Vb, vs, w.W, c->d_partial, w.h1, s, 1, w.state));
  }
  {
    ProfScope ps(c, 1, vbytes * (j + 3), 8.0 * n * q * (j + 1));
    HH_CHECK(launch_basis_update(j + 1, sg, w.Vb, vs, w.h1, w.W, c->d_partial, w.tmp, s, w.state));
  }
  HH_CHECK(launch_reorth_flag(S, j + 1, w.h1 + (size_t)(j + 1) * S, w.tmp, c->reorth_eta, w.need, w.h2, s, w.state));
  HH_CHECK(launch_multidot(j + 1, sg, w.Vb, vs, w.W, c->d_partial, w.h2, s, 0, w.need));
  HH_CHECK(launch_basis_update(j + 1, sg, w.Vb, vs, w.h2, w.W, c->d_partial, w.tmp, s, w.need));
  HH_CHECK(launch_normalize(sg, w.tmp, w.W, w.Vb + (j + 1) * vs, w.hn, s, w.state));
  HH_CHECK(launch_gmres_step(S, j, m, w.H, w.h1, w.h2, w.hn, w.cs, w.sn, w.g, w.est, w.state, w.thr, maxit, w.any, s));
  return HH_OK;
}

// Enqueues Arnoldi step j: eagerly, or (graphs on, from the second solve with
// this work space on) by replaying its captured graph, capturing it first.
hh_status run_step(hh_ctx* c, int q, int j, int maxit) {
  hh_ctx::Gmres& w = c->gw;
  const bool use = c->graphs && w.solves > 0 && c->stream != nullptr && !c->prof;
  if (!use) return arnoldi_step(c, q, j, maxit);
  if (w.epoch != c->epoch) {
    drop_graphs(c);
    w.epoch = c->epoch;
  }
  // maxit is a kernel argument of the step: graphs are kept for one value
  if ((int)w.exec.size() != w.m + 1) {
    drop_graphs(c);
    w.exec.assign(w.m + 1, nullptr);
  }
  if (c->gw_maxit != maxit) {
    drop_graphs(c);
    w.exec.assign(w.m + 1, nullptr);
    c->gw_maxit = maxit;
  }
  if (!w.exec[j]) {
    HH_CHECK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    const hh_status st = arnoldi_step(c, q, j, maxit);
    c->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (st != HH_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return device_fail(c, "hipStreamEndCapture", e);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return device_fail(c, "hipGraphInstantiate", ei);
    w.exec[j] = exec;
  }
  HH_CHECK(hipGraphLaunch(w.exec[j], c->stream));
  return HH_OK;
}

// Right-preconditioned restarted GMRES (flexible form: Z_j = B v_j kept) for
// every outer-loop system at once; q right-hand sides per problem, S systems.
hh_status gmres(hh_ctx* c, int q, const c128* b, c128* u, double rtol, int maxit, const std::vector<double>& nb,
                std::vector<int>& iters, std::vector<double>& relres, std::vector<int>& conv) {
  const long long n = c->lv[0].total;
  const SegDev& sg = c->sg;
  const int S = sg.S;
  const int m = std::max(1, std::min(c->restart, std::max(maxit, 1)));
  hipStream_t s = c->stream;
  HH_TRY(ensure_gmres(c, q, m));
  HH_TRY(ensure_partial(c, (size_t)(m + 2) * S * sg.NBmax));
  HH_TRY(ensure_poll(c));
  hh_ctx::Gmres& w = c->gw;
  c128 *Vb = w.Vb, *Zb = w.Zb, *W = w.W, *H = w.H, *g = w.g, *tmp = w.tmp, *y = w.y;
  double* thr = w.thr;
  int* state = w.state;
#define GC(expr) HH_CHECK(expr)
#define GT(expr) HH_TRY(expr)
  const long long vs = (long long)q * n;
  std::vector<double> beta(S), th(S);
  std::vector<int> hstate(3 * S);
  for (int k = 0; k < S; ++k) th[k] = rtol * nb[k];
  GC(hipMemcpyAsync(thr, th.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
  // u = 0, r = b
  GC(launch_fill_zero(u, vs * (long long)sizeof(c128), s));
  GC(launch_copy(b, W, vs, s));
  GT(norms(c, W, tmp, beta));
  int* poll = c->poll;
  while (true) {
    bool any_active = false;
    for (int k = 0; k < S; ++k) {
      relres[k] = nb[k] > 0.0 ? beta[k] / nb[k] : 0.0;
      conv[k] = relres[k] < rtol || nb[k] == 0.0;
      hstate[k] = !conv[k] && iters[k] < maxit;
      hstate[S + k] = 0;
      hstate[2 * S + k] = iters[k];
      any_active = any_active || hstate[k];
    }
    if (!any_active) break;
    // V_0 = r / beta (tmp holds ||r||^2 from norms()); g = beta e_1
    GC(launch_normalize(sg, tmp, W, Vb, nullptr, s));
    std::vector<c128> g0((size_t)S * (m + 1), make_double2(0.0, 0.0));
    for (int k = 0; k < S; ++k) g0[(size_t)k * (m + 1)] = make_double2(beta[k], 0.0);
    GC(hipMemcpyAsync(g, g0.data(), g0.size() * sizeof(c128), hipMemcpyHostToDevice, s));
    GC(hipMemcpyAsync(state, hstate.data(), 3 * S * sizeof(int), hipMemcpyHostToDevice, s));
    // the preconditioner and the Gram-Schmidt passes skip the systems that have stopped
    struct ActiveScope {
      hh_ctx* c;
      ActiveScope(hh_ctx* c_, const int* a) : c(c_) { c->act = a; }
      ~ActiveScope() { c->act = nullptr; }
    } act_scope(c, state);
    for (int j = 0; j < m; ++j) {
      GT(run_step(c, q, j, maxit));
      // poll the active count one step late so the stream never drains
      GC(hipMemcpyAsync(poll + (j & 1), w.any, sizeof(int), hipMemcpyDeviceToHost, s));
      GC(hipEventRecord(c->poll_ev[j & 1], s));
      if (j > 0) {
        GC(hipEventSynchronize(c->poll_ev[(j - 1) & 1]));
        if (poll[(j - 1) & 1] == 0) break;
      }
    }
    GC(hipMemcpyAsync(hstate.data(), state, 3 * S * sizeof(int), hipMemcpyDeviceToHost, s));
    GC(hipStreamSynchronize(s));
    for (int k = 0; k < S; ++k) iters[k] = hstate[2 * S + k];
    GC(launch_gmres_solve_small(S, m, state + S, H, g, y, s));
    GC(launch_basis_combine(sg, state + S, Zb, vs, y, u, s));
    GC(launch_apply_box(c->d_ops, c->lv[0].d, c->lv[0].nbox, c->lv[0].max_n, q, u, b, W, 1, s));
    GT(norms(c, W, tmp, beta));
  }
  w.solves += 1;
#undef GC
#undef GT
  return HH_OK;
}

hh_status stationary(hh_ctx* c, int q, const c128* b, c128* u, double rtol, int maxit, const std::vector<double>& nb,
                     std::vector<int>& iters, std::vector<double>& relres, std::vector<int>& conv) {
  const long long n = c->lv[0].total;
  const long long vs = (long long)q * n;
  const int S = c->sg.S;
  hipStream_t s = c->stream;
  c128 *r = nullptr, *z = nullptr, *tmp = nullptr;
  int* act = nullptr;
  hh_status st = HH_OK;
  auto cleanup = [&]() {
    for (void* p : std::initializer_list<void*>{r, z, tmp, act}) dfree(c, p);
  };
  if ((st = dalloc(c, &r, (size_t)vs)) != HH_OK || (st = dalloc(c, &z, (size_t)vs)) != HH_OK ||
      (st = dalloc(c, &tmp, (size_t)S)) != HH_OK || (st = dalloc(c, &act, (size_t)S)) != HH_OK) {
    cleanup();
    return st;
  }
  std::vector<double> rn(S);
  std::vector<int> active(S);
  hipError_t e;
  if ((e = launch_fill_zero(u, vs * (long long)sizeof(c128), s)) != hipSuccess ||
      (e = launch_copy(b, r, vs, s)) != hipSuccess) {
    cleanup();
    return device_fail(c, "stationary init", e);
  }
  while (true) {
    if ((st = norms(c, r, tmp, rn)) != HH_OK) break;
    bool any = false;
    for (int k = 0; k < S; ++k) {
      relres[k] = nb[k] > 0.0 ? rn[k] / nb[k] : 0.0;
      conv[k] = relres[k] < rtol || nb[k] == 0.0;
      active[k] = !conv[k] && iters[k] < maxit;
      any = any || active[k];
    }
    if (!any) break;
    if ((st = two_level(c, 0, q, r, z)) != HH_OK) break;
    if ((e = hipMemcpyAsync(act, active.data(), S * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_seg_add(c->sg, act, z, u, s)) != hipSuccess ||
        (e = launch_apply_box(c->d_ops, c->lv[0].d, c->lv[0].nbox, c->lv[0].max_n, q, u, b, r, 1, s)) != hipSuccess) {
      cleanup();
      return device_fail(c, "stationary step", e);
    }
    for (int k = 0; k < S; ++k) iters[k] += active[k];
  }
  cleanup();
  return st;
}

}  // namespace

extern "C" hh_status hh_solve(hh_ctx* c, int32_t nrhs, const void* f, const void* g, void* u, double rtol,
                              int32_t maxit, hh_solve_info* info) {
  HH_TRY(check_usable(c));
  if (nrhs <= 0 || !f || !u || maxit < 0 || !(rtol >= 0.0)) return fail(c, HH_EINVAL, "bad arguments to hh_solve");
  HH_TRY(check_built(c));
  const int q = nrhs;
  HH_TRY(ensure_work(c, 0, q));
  HH_TRY(ensure_segs(c, q));
  const int S = c->sg.S;
  Level& R0 = c->lv[0];
  const c128* b = reinterpret_cast<const c128*>(f);
  if (g) {
    // b = f + (boundary facets)/2^(dim-1) * g / h, built by the stencil kernel's rhs mode on E
    HH_CHECK(launch_rhs_with_impedance(c->d_ops, R0.d, R0.nbox, q, b, reinterpret_cast<const c128*>(g), R0.E, c->stream));
    b = R0.E;
  }
  std::vector<double> nb;
  c128* tmp = nullptr;
  HH_TRY(dalloc(c, &tmp, (size_t)S));
  hh_status st = norms(c, b, tmp, nb);
  dfree(c, tmp);
  if (st != HH_OK) return st;
  for (double v : nb)
    if (!std::isfinite(v)) return fail(c, HH_EINVAL, "right-hand side holds NaN or Inf");
  std::vector<int> iters(S, 0), conv(S, 0);
  std::vector<double> relres(S, 0.0);
  if (c->outer == HH_GMRES)
    st = gmres(c, q, b, reinterpret_cast<c128*>(u), rtol, maxit, nb, iters, relres, conv);
  else
    st = stationary(c, q, b, reinterpret_cast<c128*>(u), rtol, maxit, nb, iters, relres, conv);
  if (st != HH_OK) return st;
  if (c->prof) {
    HH_TRY(sync(c));
    prof_collect(c);
  }
  bool all = true;
  for (int k = 0; k < S; ++k) {
    if (info) {
      info[k].iters = iters[k];
      info[k].converged = conv[k];
      info[k].rel_residual = relres[k];
    }
    all = all && conv[k];
  }
  if (!all) return fail(c, HH_ENOTCONV, "not converged within maxit");
  return HH_OK;
}

extern "C" hh_status hh_profile(hh_ctx* c, int32_t enable) {
  HH_TRY(check_usable(c));
  HH_TRY(sync(c));
  prof_collect(c);
  c->prof = enable != 0;
  for (int f = 0; f < 4; ++f) {
    c->prof_ms[f] = 0.0;
    c->prof_bytes[f] = 0.0;
    c->prof_flops[f] = 0.0;
    c->prof_n[f] = 0;
  }
  return HH_OK;
}

extern "C" hh_status hh_profile_read(hh_ctx* c, int32_t family, int64_t* launches, double* total_ms, double* bytes,
                                     double* flops) {
  HH_TRY(check_usable(c));
  if (family < 0 || family > 3) return fail(c, HH_EINVAL, "unknown kernel family");
  HH_TRY(sync(c));
  prof_collect(c);
  if (launches) *launches = c->prof_n[family];
  if (total_ms) *total_ms = c->prof_ms[family];
  if (bytes) *bytes = c->prof_bytes[family];
  if (flops) *flops = c->prof_flops[family];
  return HH_OK;
}

extern "C" hh_status hh_get_coarse(hh_ctx* c, int32_t level, int32_t parent, int32_t* n_c, void* Ac_host,
                                   double* sigma_host) {
  HH_TRY(check_usable(c));
  if (level < 0 || level >= c->L) return fail(c, HH_EINVAL, "level must be in 0..levels-1");
  Level& P = c->lv[level];
  Level& Ch = c->lv[level + 1];
  if (!Ch.built) return fail(c, HH_ESTATE, "coarse space not built");
  if (parent < 0 || parent >= P.nbox) return fail(c, HH_EINVAL, "parent out of range");
  const ParentDev& pd = P.hp[parent];
  if (n_c) *n_c = pd.n_c;
  if (Ac_host && pd.n_c > 0) {
    HH_CHECK(hipMemcpyAsync(Ac_host, P.Araw + pd.aoff, (size_t)pd.n_c * pd.n_c * sizeof(c128),
                            hipMemcpyDeviceToHost, c->stream));
    HH_TRY(sync(c));
  }
  if (sigma_host) {
    size_t o = 0;
    for (int ch : c->geo.levels[level][parent].children) {
      const int sw = Ch.hb[ch].s;
      for (int t = 0; t < sw; ++t) sigma_host[o++] = Ch.sigma[(size_t)ch * Ch.smax + t];
    }
  }
  return HH_OK;
}

extern "C" hh_status hh_get_basis(hh_ctx* c, int32_t level, int32_t box, int32_t* n_own, int32_t* r_i,
                                  void* C_host) {
  HH_TRY(check_usable(c));
  if (level < 1 || level > c->L) return fail(c, HH_EINVAL, "level must be in 1..levels");
  Level& Lv = c->lv[level];
  if (!Lv.built) return fail(c, HH_ESTATE, "coarse space not built");
  if (box < 0 || box >= Lv.nbox) return fail(c, HH_EINVAL, "box out of range");
  const BoxDev& b = Lv.hb[box];
  if (n_own) *n_own = b.n_own;
  if (r_i) *r_i = b.r;
  if (C_host && b.r > 0) {
    HH_CHECK(hipMemcpyAsync(C_host, Lv.C + b.coff, (size_t)b.r * b.n_own * sizeof(c128), hipMemcpyDeviceToHost,
                            c->stream));
    HH_TRY(sync(c));
  }
  return HH_OK;
}

// ------------------------------------------------------------------ serving hooks
namespace helmdd_internal {

hh_status set_stream(hh_ctx* c, hipStream_t s) {
  if (!c) return HH_EINVAL;
  if (c->stream == s) return HH_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return HH_EDEVICE;
  c->stream = s;
  return HH_OK;
}

void release_work(hh_ctx* c) {
  if (!c) return;
  release_gmres(c);
  ++c->epoch;
  for (Level& L : c->lv) {
    for (c128** b : {&L.R, &L.X, &L.T, &L.E, &L.U, &L.cvec, &L.yvec, &L.W, &L.RP}) {
      dfree(c, *b);
      *b = nullptr;
    }
    L.qcap = 0;
    L.rp_len = 0;
  }
}

size_t resident_bytes(const hh_ctx* c) {
  size_t n = 0;
  if (c)
    for (const DevBuf& b : c->allocs) n += b.bytes;
  return n;
}

Footprint estimate_bytes(const hh_operator* A, const hh_decomposition* d, const int32_t* rank,
                         int32_t oversample, int32_t restart, int32_t precision) {
  Footprint f;
  if (!A || !d || d->levels < 1 || d->levels > 8) return f;
  Geometry g;
  if (!build_geometry(A->dim, A->n_cells, d->levels, d->m, d->overlap_cells, g).empty()) return f;
  const double c16 = 16.0;
  double op = 0.0, rhs = 0.0, work = 0.0, work_below = 0.0, smax = 1.0;
  // leaf factors: FP64 during the set-up (plus the complex64 copy when mixed)
  double gl = 0.0;
  for (const HBox& b : g.levels[g.depth()]) gl += (double)b.nx() * b.ny() * b.ny();
  op += gl * c16 + (precision == HH_MIXED ? gl * 8.0 : 0.0);
  const double n0 = (double)g.levels[0][0].n();
  for (int l = 0; l <= g.depth(); ++l) {
    double tot = 0.0, csz = 0.0, nc = 0.0;
    for (const HBox& b : g.levels[l]) {
      tot += b.n();
      if (l >= 1) {
        const double r = std::min<double>((double)rank[l - 1] * b.n_if, (double)b.iface.size());
        const double sk = std::min<double>(r + oversample, (double)b.iface.size());
        csz += r * b.n_own() + sk * b.iface.size() * 3.0;  // C, Omega / sketch blocks
        nc += r;
        smax = std::max(smax, sk);
      }
    }
    op += csz * c16 * 2.0 + nc * nc * c16 * 2.0;  // coarse blocks, Galerkin products, A_c^{-1}
    work += tot * c16 * 6.0 + nc * c16 * 2.0;     // level work buffers per column
    if (l >= 1) work_below += tot * c16 * 6.0 + nc * c16 * 2.0;
  }
  rhs = work + (2.0 * restart + 3.0) * n0 * c16;  // plus the Krylov bases V, Z and work
  f.op = (size_t)op;
  f.per_rhs = (size_t)rhs;
  f.setup = (size_t)(work_below * smax);  // the sketches run smax columns through levels 1 .. L
  return f;
}

}  // namespace helmdd_internal
