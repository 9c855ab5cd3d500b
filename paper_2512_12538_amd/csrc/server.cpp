// Serving loop: solve requests for many operators, continuously batched.
//
// Requests enter a queue.  Worker threads (one HIP stream each) take the
// oldest request whose operator is idle, together with every queued request
// for the same operator and tolerance that fits the batch width, and run them
// as one multi-right-hand-side hh_solve.  Prepared operators (leaf factors,
// coarse spaces of every level) stay cached on the device keyed by operator
// id; a miss is admitted only when its estimated footprint fits the memory
// budget, after evicting idle operators in least-recently-used order, and
// waits otherwise.  Requests arriving while batches run join the next batch
// of their operator; batches of different operators run concurrently on the
// workers' streams.  Every right-hand side gives the same bits in any batch
// (the solver's reductions do not depend on the batch), so a result does not
// depend on what it was served with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/helmdd.h"
#include "internal.h"
#include "pool.h"
#include "rng.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

struct OperatorSpec {
  hh_operator op{};
  std::vector<double> k;  // copied wavenumbers (empty: constant)
  hh_decomposition d{};
  int32_t rank[8] = {0};
  int32_t oversample = 0;
  uint64_t seed = 0;
  // estimates: prepared operator, its set-up work space, solve work space per right-hand side
  size_t op_bytes = 0, setup_bytes = 0, rhs_bytes = 0;
};

struct Entry {
  std::shared_ptr<OperatorSpec> spec;
  hh_ctx* ctx = nullptr;
  size_t bytes = 0;      // resident bytes once prepared
  size_t reserved = 0;   // bytes counted against the budget
  bool busy = false;
  Clock::time_point last;
};

struct Request {
  uint64_t ticket = 0;
  uint64_t id = 0;
  int32_t nrhs = 0;
  const void* f = nullptr;
  void* u = nullptr;
  double rtol = 0.0;
  int32_t maxit = 0;
  Clock::time_point submit, start;
  bool done = false;
  hh_request_result res{};
};

bool same_shape(const OperatorSpec& a, const hh_request& r) {
  if (a.op.dim != r.op.dim || a.op.n_cells != r.op.n_cells) return false;
  if (a.d.levels != r.decomposition.levels) return false;
  for (int l = 0; l < a.d.levels; ++l)
    if (a.d.m[l][0] != r.decomposition.m[l][0] || a.d.m[l][1] != r.decomposition.m[l][1] ||
        a.d.overlap_cells[l] != r.decomposition.overlap_cells[l] || a.rank[l] != r.rank_per_interface[l])
      return false;
  return a.oversample == r.oversample;
}

}  // namespace

struct hh_server {
  hh_server_options o{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> requests;  // by ticket
  std::map<uint64_t, Entry> cache;                        // by operator id
  std::map<uint64_t, std::shared_ptr<OperatorSpec>> specs;
  size_t used = 0;  // reserved device bytes (operators + running batches)
  int preparing = 0;  // workers setting up a new operator
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  long long served = 0, misses = 0, evictions = 0;
  std::string last_err;  // message of the last failed batch

  void worker(int w);
  bool take_batch(std::unique_lock<std::mutex>& lk, std::vector<Request*>& batch, uint64_t& id);
  hh_status prepare(Entry& e, hipStream_t s);
};

// Oldest queued request whose operator is idle, plus the queued requests of
// that operator and tolerance that fit the batch width (arrival order).  A
// request for an operator not yet prepared is passed over while all other
// workers are already preparing operators, so that prepared operators keep
// being served.  The batch width is capped so that its work space takes at
// most half the budget.
bool hh_server::take_batch(std::unique_lock<std::mutex>&, std::vector<Request*>& batch, uint64_t& id) {
  for (auto it = queue.begin(); it != queue.end(); ++it) {
    Request* r = *it;
    auto ce = cache.find(r->id);
    if (ce != cache.end() && ce->second.busy) continue;
    const bool miss = ce == cache.end() || !ce->second.ctx;
    if (miss && o.workers > 1 && preparing >= o.workers - 1) continue;
    OperatorSpec& sp = *specs[r->id];
    if (sp.rhs_bytes == 0) {
      const helmdd_internal::Footprint fp =
          helmdd_internal::estimate_bytes(&sp.op, &sp.d, sp.rank, sp.oversample, o.gmres_restart, o.precision);
      sp.op_bytes = fp.op;
      sp.setup_bytes = fp.setup;
      sp.rhs_bytes = std::max<size_t>(fp.per_rhs, 1);
    }
    const long long cap = std::max<long long>(1, (long long)(o.budget_bytes / 2) / (long long)sp.rhs_bytes);
    const int wmax = (int)std::min<long long>(o.max_batch_rhs, std::max<long long>(cap, r->nrhs));
    id = r->id;
    int width = 0;
    for (auto jt = it; jt != queue.end();) {
      Request* x = *jt;
      if (x->id == id && x->rtol == r->rtol && x->maxit == r->maxit && width + x->nrhs <= wmax) {
        width += x->nrhs;
        batch.push_back(x);
        jt = queue.erase(jt);
      } else {
        ++jt;
      }
    }
    return true;
  }
  return false;
}

hh_status hh_server::prepare(Entry& e, hipStream_t s) {
  const OperatorSpec& sp = *e.spec;
  hh_operator op = sp.op;
  op.k = sp.k.empty() ? nullptr : sp.k.data();
  hh_options opt{};
  opt.precision = o.precision;
  opt.outer = HH_GMRES;
  opt.gmres_restart = o.gmres_restart;
  opt.stream = s;
  hh_ctx* c = nullptr;
  hh_status st = hh_setup(&op, &sp.d, &opt, &c);
  if (st != HH_OK) return st;
  std::vector<double> host;
  void* dom = nullptr;
  size_t dom_bytes = 0;
  for (int level = sp.d.levels; level >= 1 && st == HH_OK; --level) {
    const int rank = sp.rank[level - 1];
    int32_t nb = 0;
    st = hh_level_info(c, level, rank, sp.oversample, &nb, nullptr, nullptr, nullptr);
    if (st != HH_OK) break;
    std::vector<int32_t> m_in(nb), ss(nb);
    st = hh_level_info(c, level, rank, sp.oversample, nullptr, m_in.data(), nullptr, ss.data());
    if (st != HH_OK) break;
    if (rank == 0) {
      st = hh_build_coarse(c, level, 0, sp.oversample, nullptr);
      continue;
    }
    size_t total = 0;
    for (int i = 0; i < nb; ++i) total += (size_t)m_in[i] * ss[i];
    host.assign(2 * total, 0.0);
    size_t off = 0;
    for (int i = 0; i < nb; ++i) {
      // the block of box i, sample-major (s x m_in), is the column-major m_in x s layout of hh_build_coarse
      rng::omega_block(sp.seed, level, i, m_in[i], ss[i], host.data() + 2 * off);
      off += (size_t)m_in[i] * ss[i];
    }
    const size_t need = 16 * std::max<size_t>(total, 1);
    if (need > dom_bytes) {
      if (dom) devpool::release(dom, dom_bytes, s);
      dom = devpool::acquire(need, s);
      dom_bytes = need;
      if (!dom) {
        st = HH_ENOMEM;
        break;
      }
    }
    if (hipMemcpyAsync(dom, host.data(), 16 * total, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = HH_EDEVICE;
      break;
    }
    st = hh_build_coarse(c, level, rank, sp.oversample, dom);
  }
  if (dom) devpool::release(dom, dom_bytes, s);
  if (st != HH_OK) {
    hh_destroy(c);
    return st;
  }
  helmdd_internal::release_work(c);  // cached operators keep factors and coarse data only
  e.ctx = c;
  e.bytes = helmdd_internal::resident_bytes(c);
  return HH_OK;
}

void hh_server::worker(int w) {
  (void)hipSetDevice(device);
  hipStream_t s = streams[w];
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    std::vector<Request*> batch;
    uint64_t id = 0;
    while (!stop && !take_batch(lk, batch, id)) cv.wait(lk);
    if (stop && batch.empty()) return;
    Entry& e = cache[id];
    if (!e.spec) e.spec = specs[id];
    e.busy = true;
    const OperatorSpec& sp = *e.spec;
    int q = 0;
    for (Request* r : batch) q += r->nrhs;
    const bool hit = e.ctx != nullptr;
    // admission: the operator (on a miss) and this batch's work space; the
    // set-up work space is returned before the solve's is taken
    const size_t est_run = sp.rhs_bytes * (size_t)q;
    const size_t est_op = hit ? 0 : sp.op_bytes + (sp.setup_bytes > est_run ? sp.setup_bytes - est_run : 0);
    const size_t need = est_op + est_run;
    hh_status st = HH_OK;
    std::string reason;  // admission failures
    bool charged = false;
    while (used + need > (size_t)o.budget_bytes) {
      // evict the least recently used idle operator
      auto victim = cache.end();
      for (auto it = cache.begin(); it != cache.end(); ++it)
        if (!it->second.busy && it->second.ctx && (victim == cache.end() || it->second.last < victim->second.last))
          victim = it;
      if (victim != cache.end()) {
        hh_ctx* vc = victim->second.ctx;
        used -= victim->second.reserved;
        cache.erase(victim);
        ++evictions;
        lk.unlock();
        hh_destroy(vc);
        lk.lock();
        continue;
      }
      bool others = false;
      for (auto& kv : cache)
        if (kv.first != id && kv.second.busy) others = true;
      if (!others) {
        st = HH_ENOMEM;  // does not fit even alone
        reason = "the operator and the batch's work space do not fit in the budget";
        break;
      }
      if (stop) {
        st = HH_ESTATE;
        reason = "server stopping";
        break;
      }
      cv.wait(lk);  // memory frees when another batch ends
    }
    if (st == HH_OK) {
      used += need;
      charged = true;
      if (!hit) ++preparing;
    }
    const Clock::time_point t_start = Clock::now();
    for (Request* r : batch) r->start = t_start;
    lk.unlock();

    if (st == HH_OK && !hit) {
      st = prepare(e, s);
      lk.lock();
      ++misses;
      // keep the measured footprint reserved instead of the estimate
      used -= est_op;
      --preparing;
      if (st == HH_OK) {
        used += e.bytes;
        e.reserved = e.bytes;
      }
      lk.unlock();
    }
    if (st == HH_OK) st = helmdd_internal::set_stream(e.ctx, s);
    std::vector<hh_solve_info> info(q);
    if (st == HH_OK) {
      const long long nodes = sp.op.dim == 2 ? (long long)(sp.op.n_cells + 1) * (sp.op.n_cells + 1)
                                             : (long long)(sp.op.n_cells + 1);
      const size_t vb = (size_t)q * nodes * 16;
      void* F = devpool::acquire(vb, s);
      void* U = devpool::acquire(vb, s);
      if (!F || !U) {
        st = HH_ENOMEM;
        reason = "no device memory for the batch's right-hand sides";
      } else {
        size_t off = 0;
        for (Request* r : batch) {
          const size_t b = (size_t)r->nrhs * nodes * 16;
          if (hipMemcpyAsync((char*)F + off, r->f, b, hipMemcpyDeviceToDevice, s) != hipSuccess) st = HH_EDEVICE;
          off += b;
        }
        if (st == HH_OK) {
          st = hh_solve(e.ctx, q, F, nullptr, U, batch.front()->rtol, batch.front()->maxit, info.data());
          if (st == HH_ENOTCONV) st = HH_OK;  // reported per request below
        }
        if (st == HH_OK) {
          off = 0;
          for (Request* r : batch) {
            const size_t b = (size_t)r->nrhs * nodes * 16;
            if (hipMemcpyAsync(r->u, (char*)U + off, b, hipMemcpyDeviceToDevice, s) != hipSuccess) st = HH_EDEVICE;
            off += b;
          }
          if (hipStreamSynchronize(s) != hipSuccess) st = HH_EDEVICE;
        }
        helmdd_internal::release_work(e.ctx);
      }
      if (F) devpool::release(F, vb, s);
      if (U) devpool::release(U, vb, s);
    }
    const Clock::time_point t_end = Clock::now();
    std::string msg;
    if (st != HH_OK) {
      const char* why = !reason.empty() ? reason.c_str()
                        : e.ctx       ? hh_last_error(e.ctx)
                                      : hh_last_error(nullptr);  // set-up failures: this thread's
      msg = std::string(hh_status_string(st)) + " (operator " + std::to_string(id) + ", " + std::to_string(q) +
            " rhs): " + why;
      const hipError_t he = hipGetLastError();
      if (he != hipSuccess) msg += std::string(" [HIP: ") + hipGetErrorString(he) + "]";
    }

    lk.lock();
    if (!msg.empty()) last_err = msg;
    if (charged) used -= est_run;
    int col = 0;
    for (Request* r : batch) {
      hh_request_result& res = r->res;
      res.status = st;
      res.iters = 0;
      res.rel_residual = 0.0;
      if (st == HH_OK) {
        bool conv = true;
        for (int t = 0; t < r->nrhs; ++t) {
          res.iters = std::max(res.iters, info[col + t].iters);
          res.rel_residual = std::max(res.rel_residual, info[col + t].rel_residual);
          conv = conv && info[col + t].converged;
        }
        if (!conv) res.status = HH_ENOTCONV;
      }
      col += r->nrhs;
      res.latency_s = seconds(r->submit, t_end);
      res.queue_s = seconds(r->submit, r->start);
      res.batch_rhs = q;
      res.cache_hit = hit ? 1 : 0;
      r->done = true;
      ++served;
    }
    e.busy = false;
    e.last = t_end;
    if (!e.ctx) cache.erase(id);  // failed preparation: nothing cached
    cv.notify_all();
  }
}

extern "C" {

hh_status hh_server_create(const hh_server_options* o, hh_server** out) {
  if (!o || !out) return HH_EINVAL;
  *out = nullptr;
  if (o->budget_bytes <= 0 || o->workers < 1 || o->workers > 16 || o->max_batch_rhs < 1 ||
      (o->precision != HH_FP64 && o->precision != HH_MIXED) || o->gmres_restart < 0 || o->gmres_restart > 120)
    return HH_EINVAL;
  hh_server* sv = new (std::nothrow) hh_server;
  if (!sv) return HH_ENOMEM;
  sv->o = *o;
  if (sv->o.gmres_restart == 0) sv->o.gmres_restart = 50;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return HH_EDEVICE;
  }
  for (int w = 0; w < o->workers; ++w) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : sv->streams) (void)hipStreamDestroy(t);
      delete sv;
      return HH_EDEVICE;
    }
    sv->streams.push_back(s);
  }
  for (int w = 0; w < o->workers; ++w) sv->workers.emplace_back(&hh_server::worker, sv, w);
  *out = sv;
  return HH_OK;
}

hh_status hh_server_submit(hh_server* sv, const hh_request* r, uint64_t* ticket) {
  if (!sv || !r || !ticket) return HH_EINVAL;
  if (r->nrhs < 1 || r->nrhs > sv->o.max_batch_rhs || !r->f || !r->u || r->maxit < 1 || !(r->rtol >= 0.0))
    return HH_EINVAL;
  if (r->op.dim != 1 && r->op.dim != 2) return HH_EINVAL;
  if (r->decomposition.levels < 1 || r->decomposition.levels > 8) return HH_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto sp = sv->specs.find(r->operator_id);
  if (sp == sv->specs.end()) {
    auto spec = std::make_shared<OperatorSpec>();
    spec->op = r->op;
    if (r->op.k) {
      const size_t n = r->op.dim == 2 ? (size_t)(r->op.n_cells + 1) * (r->op.n_cells + 1) : (size_t)r->op.n_cells + 1;
      spec->k.assign(r->op.k, r->op.k + n);
    }
    spec->op.k = nullptr;
    spec->d = r->decomposition;
    std::memcpy(spec->rank, r->rank_per_interface, sizeof(spec->rank));
    spec->oversample = r->oversample;
    spec->seed = r->omega_seed;
    sv->specs[r->operator_id] = spec;
  } else if (!same_shape(*sp->second, *r)) {
    return HH_EINVAL;  // one id, one operator
  }
  auto req = std::make_unique<Request>();
  req->ticket = sv->next_ticket++;
  req->id = r->operator_id;
  req->nrhs = r->nrhs;
  req->f = r->f;
  req->u = r->u;
  req->rtol = r->rtol;
  req->maxit = r->maxit;
  req->submit = Clock::now();
  *ticket = req->ticket;
  sv->queue.push_back(req.get());
  sv->requests[req->ticket] = std::move(req);
  sv->cv.notify_all();
  return HH_OK;
}

hh_status hh_server_wait(hh_server* sv, uint64_t ticket, double timeout_s, hh_request_result* res) {
  if (!sv) return HH_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->requests.find(ticket);
  if (it == sv->requests.end()) return HH_EINVAL;
  Request* r = it->second.get();
  const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                        std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s));
  while (!r->done)
    if (sv->cv.wait_until(lk, until) == std::cv_status::timeout && !r->done) return HH_ESTATE;
  if (res) *res = r->res;
  sv->requests.erase(it);  // a result is handed out once
  return HH_OK;
}

hh_status hh_server_stats(hh_server* sv, int64_t* served, int64_t* misses, int64_t* evictions, int64_t* cached,
                          int64_t* reserved_bytes) {
  if (!sv) return HH_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (served) *served = sv->served;
  if (misses) *misses = sv->misses;
  if (evictions) *evictions = sv->evictions;
  if (cached) *cached = (int64_t)sv->cache.size();
  if (reserved_bytes) *reserved_bytes = (int64_t)sv->used;
  return HH_OK;
}

const char* hh_server_last_error(hh_server* sv) {
  thread_local std::string copy;
  if (!sv) return "null server";
  std::lock_guard<std::mutex> lk(sv->mu);
  copy = sv->last_err;
  return copy.c_str();
}

hh_status hh_server_destroy(hh_server* sv) {
  if (!sv) return HH_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->queue.clear();  // requests not yet started are dropped
  }
  sv->cv.notify_all();
  for (std::thread& t : sv->workers) t.join();
  for (auto& kv : sv->cache)
    if (kv.second.ctx) hh_destroy(kv.second.ctx);
  for (hipStream_t s : sv->streams) {
    devpool::forget_stream(s);  // no cached block may keep an event of a destroyed stream
    (void)hipStreamDestroy(s);
  }
  delete sv;
  (void)hipGetLastError();  // clean-up ignores errors; leave none behind for the caller's next call
  return HH_OK;
}

hh_status hh_estimate_device_bytes(const hh_operator* A, const hh_decomposition* d, const int32_t* rank,
                                   int32_t oversample, int32_t nrhs, int32_t gmres_restart, int32_t precision,
                                   int64_t* bytes) {
  if (!A || !d || !rank || !bytes || nrhs < 0) return HH_EINVAL;
  const helmdd_internal::Footprint f =
      helmdd_internal::estimate_bytes(A, d, rank, oversample, gmres_restart > 0 ? gmres_restart : 50, precision);
  if (f.op == 0) return HH_EINVAL;
  *bytes = (int64_t)(f.op + std::max(f.setup, f.per_rhs * (size_t)nrhs));
  return HH_OK;
}

hh_status hh_omega_philox(uint64_t seed, int32_t level, int32_t box, int32_t m_in, int32_t s, double* out) {
  if (!out || m_in < 0 || s < 0) return HH_EINVAL;
  rng::omega_block(seed, level, box, m_in, s, out);
  return HH_OK;
}

}  // extern "C"
