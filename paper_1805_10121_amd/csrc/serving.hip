// Serving: continuous batching of many concurrent solves (sequences of correlated problems of
// uneven order, Sec. 2 and Sec. 6.1) on one device.
//
//   Batcher  -- every solve that reaches its FILTER phase hands the products of its filter
//               call (Alg. 4) to the batcher of its size class; each tick takes the next
//               product of every submitted filter and runs them all in one grouped launch per
//               product kind (FP64 or FP32, 4M on H or 3M on a planar copy).  New filter calls
//               join at the next tick.  At most two ticks are in flight, so a newly arrived
//               solve waits at most about two product times.  Solves of different orders go to
//               different batchers (own thread and stream), so the products of a small solve
//               never wait for a tick that holds the product of a much larger one; the classes'
//               launches share the device concurrently.  A product with few tiles is split
//               along K inside its grouped launch (a deterministic split that depends only on
//               its order and width), so a lone small product still fills the device.
//   Server   -- worker threads, each with its own context (HIP stream, rocBLAS handle,
//               workspace), take requests first-come first-served subject to (a) problems of
//               one sequence run in submission order, each warm-started from the previous
//               solution held in device memory, and (b) the device memory the request needs
//               fitting in the budget.  Everything outside the filter runs on the worker's own
//               stream, so the solves overlap on the device.
//
// A product is computed by the grouped kernel exactly as it would be alone (data-parallel
// tiles, fixed K order), and everything else a solve does depends only on its own data, so a
// request's results are bitwise the same whatever else is in flight.

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.h"

namespace chase {

struct Batcher::Job {
  int kind;  // 0 complex128, 1 complex64 interleaved H, 2 complex64 planar H (3M),
            // 3 complex128 planar H (3M)
  const void* H;
  int64_t ldh, n, ld;
  void* V;
  void* W;
  const std::vector<FilterProduct>* prods;
  size_t next = 0;
  hipEvent_t ready = nullptr, done = nullptr;
  bool launched = false;
  hipError_t err = hipSuccess;
};

struct Batcher::Impl {
  int device = 0;
  hipStream_t stream = nullptr;
  GroupScratch gs;  // partial sums of K-sliced grouped products (reused launch after launch)
  hipEvent_t tick_ev[2] = {nullptr, nullptr};
  bool tick_recorded[2] = {false, false};
  int tick = 0;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<Job*> incoming;
  std::vector<Job*> active;
  bool stop = false;
  int64_t launches = 0, products = 0;

  void loop();
  hipError_t tick_once();
};

size_t Batcher::scratch_bytes() { return 4 * group_scratch_min_bytes(); }

Batcher::Batcher(int device) {
  impl_ = new Impl();
  impl_->device = device;
  impl_->gs.bytes = scratch_bytes();
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&impl_->stream) != hipSuccess ||
      hipEventCreateWithFlags(&impl_->tick_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&impl_->tick_ev[1], hipEventDisableTiming) != hipSuccess ||
      hipDeviceGetAttribute(&impl_->gs.cus, hipDeviceAttributeMultiprocessorCount, device) !=
          hipSuccess ||
      hipMalloc(&impl_->gs.ptr, impl_->gs.bytes) != hipSuccess) {
    impl_->gs.ptr = nullptr;
    (void)hipGetLastError();
    return;
  }
  impl_->th = std::thread([this] { impl_->loop(); });
  ok_ = true;
}

Batcher::~Batcher() {
  if (impl_->th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(impl_->mu);
      impl_->stop = true;
    }
    impl_->cv.notify_all();
    impl_->th.join();
  }
  (void)hipSetDevice(impl_->device);
  if (impl_->stream) (void)hipStreamSynchronize(impl_->stream);
  for (auto& e : impl_->tick_ev)
    if (e) (void)hipEventDestroy(e);
  if (impl_->stream) (void)hipStreamDestroy(impl_->stream);
  if (impl_->gs.ptr) (void)hipFree(impl_->gs.ptr);
  delete impl_;
}

void Batcher::counters(int64_t* launches, int64_t* products) const {
  std::lock_guard<std::mutex> lk(impl_->mu);
  if (launches) *launches = impl_->launches;
  if (products) *products = impl_->products;
}

hipError_t Batcher::run(int kind, const void* H, int64_t ldh, int64_t n, void* V, void* W,
                        int64_t ld, const std::vector<FilterProduct>& prods, hipStream_t caller,
                        hipEvent_t ready, hipEvent_t done) {
  if (prods.empty()) return hipSuccess;
  Job job;
  job.kind = kind;
  job.H = H;
  job.ldh = ldh;
  job.n = n;
  job.ld = ld;
  job.V = V;
  job.W = W;
  job.prods = &prods;
  job.ready = ready;
  job.done = done;
  hipError_t e = hipEventRecord(job.ready, caller);
  if (e != hipSuccess) return e;
  {
    std::unique_lock<std::mutex> lk(impl_->mu);
    impl_->incoming.push_back(&job);
    impl_->cv.notify_all();
    impl_->done_cv.wait(lk, [&] { return job.launched; });
  }
  // The batcher has issued its wait on `ready` and recorded `done`, so both events may be
  // recorded again by the next call.
  if (job.err == hipSuccess) job.err = hipStreamWaitEvent(caller, job.done, 0);
  return job.err;
}

hipError_t Batcher::Impl::tick_once() {
  // keep at most two ticks in flight
  const int slot = tick & 1;
  if (tick_recorded[slot]) {
    hipError_t e = hipEventSynchronize(tick_ev[slot]);
    if (e != hipSuccess) return e;
  }
  std::vector<GroupDesc<double>> d64, d3m64;
  std::vector<GroupDesc<float>> d32, d3m;
  for (Job* j : active) {
    const FilterProduct& p = (*j->prods)[j->next];
    if (j->kind == 0 || j->kind == 3) {
      const double* V = static_cast<const double*>(j->V);
      const double* W = static_cast<const double*>(j->W);
      GroupDesc<double> d{};
      d.H = static_cast<const double*>(j->H);
      d.X = (p.from_v ? V : W) + 2 * p.col0 * j->ld;
      d.OUT = const_cast<double*>((p.from_v ? W : V) + 2 * p.col0 * j->ld);
      d.ldh = j->ldh;
      d.ldx = d.ldo = j->ld;
      d.n = static_cast<int>(j->n);
      d.ncols = static_cast<int>(p.ncols);
      d.alpha = p.alpha;
      d.beta = p.beta;
      d.gamma = p.gamma;
      (j->kind == 3 ? d3m64 : d64).push_back(d);
    } else {
      const float* V = static_cast<const float*>(j->V);
      const float* W = static_cast<const float*>(j->W);
      GroupDesc<float> d{};
      d.H = static_cast<const float*>(j->H);
      d.X = (p.from_v ? V : W) + 2 * p.col0 * j->ld;
      d.OUT = const_cast<float*>((p.from_v ? W : V) + 2 * p.col0 * j->ld);
      d.ldh = j->ldh;
      d.ldx = d.ldo = j->ld;
      d.n = static_cast<int>(j->n);
      d.ncols = static_cast<int>(p.ncols);
      d.alpha = static_cast<float>(p.alpha);
      d.beta = static_cast<float>(p.beta);
      d.gamma = static_cast<float>(p.gamma);
      (j->kind == 2 ? d3m : d32).push_back(d);
    }
    ++j->next;
  }
  hipError_t e = hipSuccess;
  if (!d64.empty())
    e = launch_hemm_group<double>(d64.data(), static_cast<int>(d64.size()), gs, stream);
  if (e == hipSuccess && !d32.empty())
    e = launch_hemm_group<float>(d32.data(), static_cast<int>(d32.size()), gs, stream);
  if (e == hipSuccess && !d3m.empty())
    e = launch_hemm_group_3m(d3m.data(), static_cast<int>(d3m.size()), gs, stream);
  if (e == hipSuccess && !d3m64.empty())
    e = launch_hemm_group_3m_f64(d3m64.data(), static_cast<int>(d3m64.size()), gs, stream);
  if (e == hipSuccess) e = hipEventRecord(tick_ev[slot], stream);
  tick_recorded[slot] = true;
  ++tick;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto nl = [](size_t c) { return static_cast<int64_t>((c + kMaxGroup - 1) / kMaxGroup); };
    launches += nl(d64.size()) + nl(d32.size()) + nl(d3m.size()) + nl(d3m64.size());
    products += static_cast<int64_t>(d64.size() + d32.size() + d3m.size() + d3m64.size());
  }
  return e;
}

void Batcher::Impl::loop() {
  (void)hipSetDevice(device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !incoming.empty() || !active.empty(); });
      if (stop && incoming.empty() && active.empty()) return;
      while (!incoming.empty()) {
        Job* j = incoming.front();
        incoming.pop_front();
        j->err = hipStreamWaitEvent(stream, j->ready, 0);
        active.push_back(j);
      }
    }
    hipError_t e = tick_once();
    std::vector<Job*> keep;
    bool any_done = false;
    for (Job* j : active) {
      if (e != hipSuccess && j->err == hipSuccess) j->err = e;
      if (j->next >= j->prods->size() || j->err != hipSuccess) {
        hipError_t r = hipEventRecord(j->done, stream);
        if (j->err == hipSuccess) j->err = r;
        any_done = true;
        std::lock_guard<std::mutex> lk(mu);
        j->launched = true;
      } else {
        keep.push_back(j);
      }
    }
    active.swap(keep);
    if (any_done) done_cv.notify_all();
  }
}

}  // namespace chase

// ------------------------------------------------------------------------------- server

struct chase_server {
  int device = 0;
  size_t budget = 0;
  // one batcher per size class: orders below 3000, 6000, 12000, and the rest
  static constexpr int kClasses = 4;
  std::unique_ptr<chase::Batcher> batchers[kClasses];
  std::vector<std::thread> workers;
  std::vector<size_t> worker_ws;  // workspace bytes each worker's context holds
  std::mutex mu;
  std::condition_variable cv, done_cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  // fixed allocations (batcher scratch, each worker's product scratch and a handle allowance)
  // + sequence states + worker workspaces
  size_t used = 0;
  size_t fixed = 0;  // the fixed part of used
  std::string last_error;

  chase::Batcher* batcher_for(int64_t n) {
    const int c = n < 3000 ? 0 : n < 6000 ? 1 : n < 12000 ? 2 : 3;
    return batchers[c].get();
  }

  struct Req {
    uint64_t seq = 0;
    chase_config cfg{};
    const void* H = nullptr;
    int64_t ldh = 0;
    bool done = false;
    int status = 0;
    std::string err;
    std::vector<double> ritzv, resid;
    chase_stats stats{};
    std::chrono::steady_clock::time_point t_submit, t_start, t_end;
  };
  std::map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;

  struct Seq {
    chase_config cfg{};
    double* V = nullptr;
    std::vector<double> ritzv;
    int64_t solved = 0;
    bool busy = false;
    size_t state_bytes = 0;
  };
  std::map<uint64_t, Seq> seqs;

  void worker(int w);
};

namespace {

size_t state_bytes_of(const chase_config& c) {
  return static_cast<size_t>(c.n) * static_cast<size_t>(c.nev + c.nex) *
         chase::solve_elem_bytes(c);
}

size_t ws_bytes_of(const chase_config& c, bool warm) {
  chase_config x = c;
  x.approx = warm ? 1 : c.approx;
  return chase_workspace_bytes(&x);
}

}  // namespace

void chase_server::worker(int w) {
  chase_ctx* ctx = nullptr;
  if (chase_create(&ctx, device, nullptr) != CHASE_OK) {
    std::lock_guard<std::mutex> lk(mu);
    last_error = "worker context creation failed";
    return;
  }
  for (;;) {
    uint64_t ticket = 0;
    Req* req = nullptr;
    Seq* seq = nullptr;
    bool fresh = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stop && queue.empty()) {
          lk.unlock();
          chase_destroy(ctx);
          return;
        }
        // first queued request whose sequence is idle and whose memory fits
        for (auto it = queue.begin(); it != queue.end(); ++it) {
          Req& r = reqs[*it];
          auto sit = seqs.find(r.seq);
          const bool exists = sit != seqs.end();
          if (exists && sit->second.busy) continue;
          const bool warm = exists && sit->second.solved > 0;
          const size_t need_ws = ws_bytes_of(r.cfg, warm);
          const size_t grow = need_ws > worker_ws[w] ? need_ws - worker_ws[w] : 0;
          const size_t extra = grow + (exists ? 0 : state_bytes_of(r.cfg));
          if (used + extra > budget) continue;
          used += extra;
          worker_ws[w] += grow;
          ticket = *it;
          queue.erase(it);
          req = &r;
          if (!exists) {
            Seq s;
            s.cfg = r.cfg;
            s.state_bytes = state_bytes_of(r.cfg);
            seqs[r.seq] = s;
            fresh = true;
          }
          seq = &seqs[r.seq];
          seq->busy = true;
          break;
        }
        if (req) break;
        cv.wait(lk);
      }
    }
    req->t_start = std::chrono::steady_clock::now();
    const int64_t nb = req->cfg.nev + req->cfg.nex;
    int rc = CHASE_OK;
    std::string err;
    if (fresh) {
      hipError_t e = hipSetDevice(device);
      if (e == hipSuccess) e = hipMalloc(&seq->V, state_bytes_of(req->cfg));
      if (e == hipSuccess)
        e = chase::launch_start_block(seq->V, req->cfg, req->cfg.seed ^ 0x5eedULL, ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        if (seq->V) (void)hipFree(seq->V);
        seq->V = nullptr;
        rc = CHASE_ENOMEM;
        err = std::string("sequence state: ") + hipGetErrorString(e);
      }
      seq->ritzv.assign(nb, 0.0);
    }
    std::vector<double> rv(nb, 0.0), rs(nb, 0.0);
    chase_stats st{};
    if (rc == CHASE_OK) {
      chase_config cfg = req->cfg;
      cfg.approx = seq->solved > 0 ? 1 : req->cfg.approx;
      if (cfg.approx) {
        cfg.have_mu = 0;
        rv = seq->ritzv;
      }
      rc = chase::solve_with(ctx, &cfg, req->H, req->ldh, seq->V, cfg.n, rv.data(), rs.data(), &st,
                             batcher_for(cfg.n));
      if (rc < 0) err = chase_last_error(ctx);
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      req->t_end = std::chrono::steady_clock::now();
      req->status = rc;
      req->err = err;
      req->ritzv = rv;
      req->resid = rs;
      req->stats = st;
      req->done = true;
      seq->busy = false;
      if (rc >= 0) {
        seq->ritzv = rv;
        ++seq->solved;
      }
      // charge what the workspace really holds (a failed growth frees the old one)
      used = used - worker_ws[w] + ctx->ws_bytes;
      worker_ws[w] = ctx->ws_bytes;
      if (!seq->V) {  // the sequence state could not be allocated: forget the sequence
        used -= seq->state_bytes;
        seqs.erase(req->seq);
      }
      (void)ticket;
    }
    done_cv.notify_all();
    cv.notify_all();
  }
}

using namespace chase;

extern "C" {

int chase_server_create(chase_server** out, int device, size_t mem_budget_bytes, int workers) {
  if (!out) return CHASE_EINVAL;
  *out = nullptr;
  if (workers < 1 || workers > 64 || mem_budget_bytes == 0) return CHASE_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return CHASE_EDEVICE;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    (void)hipGetLastError();
    return CHASE_EDEVICE;
  }
  // fixed device memory: the batchers' scratch, and per worker context its product scratch
  // plus an allowance for the rocBLAS/rocSOLVER handle workspace
  constexpr size_t kHandleAllowance = size_t{64} << 20;
  const size_t fixed = chase_server::kClasses * Batcher::scratch_bytes() +
                       static_cast<size_t>(workers) * (product_scratch_bytes(cus) + kHandleAllowance);
  if (fixed >= mem_budget_bytes) return CHASE_EINVAL;
  auto* s = new chase_server();
  s->device = device;
  s->budget = mem_budget_bytes;
  s->used = fixed;
  s->fixed = fixed;
  for (auto& b : s->batchers) {
    b.reset(new Batcher(device));
    if (!b->ok()) {
      delete s;
      return CHASE_EDEVICE;
    }
  }
  s->worker_ws.assign(workers, 0);
  for (int w = 0; w < workers; ++w) s->workers.emplace_back([s, w] { s->worker(w); });
  *out = s;
  return CHASE_OK;
}

int chase_server_submit(chase_server* s, uint64_t seq_id, const chase_config* cfg, const void* H,
                        int64_t ldh, uint64_t* ticket) {
  if (!s || !cfg || !ticket) return CHASE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->last_error.clear();
  if (check_config(nullptr, cfg) != CHASE_OK) {
    s->last_error = "invalid configuration";
    return CHASE_EINVAL;
  }
  if (!H || ldh < cfg->n) {
    s->last_error = "NULL H or ldh < n";
    return CHASE_EINVAL;
  }
  // the resident state is n x (nev+nex) elements of one type: sizes and element type are fixed
  // for the life of a sequence
  auto same_state = [&](const chase_config& c) {
    return c.n == cfg->n && c.nev == cfg->nev && c.nex == cfg->nex &&
           c.real_symmetric == cfg->real_symmetric &&
           solve_scalar_bytes(c) == solve_scalar_bytes(*cfg);
  };
  const char* kStateMsg =
      "n, nev, nex, real_symmetric and the element precision must stay the same within a sequence";
  auto sit = s->seqs.find(seq_id);
  if (sit != s->seqs.end() && !same_state(sit->second.cfg)) {
    s->last_error = kStateMsg;
    return CHASE_EINVAL;
  }
  for (uint64_t t : s->queue) {
    const auto& r = s->reqs[t];
    if (r.seq == seq_id && !same_state(r.cfg)) {
      s->last_error = kStateMsg;
      return CHASE_EINVAL;
    }
  }
  const size_t need = ws_bytes_of(*cfg, false) + state_bytes_of(*cfg);
  if (need > s->budget - s->fixed) {
    s->last_error = "request needs " + std::to_string(need) +
                    " bytes, above the budget left beside the server's fixed allocations";
    return CHASE_EBUSY;
  }
  chase_server::Req r;
  r.seq = seq_id;
  r.cfg = *cfg;
  r.H = H;
  r.ldh = ldh;
  r.t_submit = std::chrono::steady_clock::now();
  const uint64_t t = s->next_ticket++;
  s->reqs[t] = r;
  s->queue.push_back(t);
  *ticket = t;
  s->cv.notify_all();
  return CHASE_OK;
}

int chase_server_poll(chase_server* s, uint64_t ticket, int wait, int* done, double* ritzv,
                      double* resid, chase_stats* stats, double* latency_s) {
  if (!s || !done) return CHASE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    s->last_error = "unknown ticket";
    return CHASE_EINVAL;
  }
  if (wait) s->done_cv.wait(lk, [&] { return it->second.done; });
  *done = it->second.done ? 1 : 0;
  if (!*done) return CHASE_OK;
  chase_server::Req& r = it->second;
  if (ritzv) std::copy(r.ritzv.begin(), r.ritzv.end(), ritzv);
  if (resid) std::copy(r.resid.begin(), r.resid.end(), resid);
  if (stats) *stats = r.stats;
  if (latency_s)
    *latency_s = std::chrono::duration<double>(r.t_end - r.t_submit).count();
  const int status = r.status;
  if (status < 0) s->last_error = r.err;
  s->reqs.erase(it);
  return status;
}

int chase_server_vectors(chase_server* s, uint64_t seq_id, void** V, int64_t* ldv) {
  if (!s || !V || !ldv) return CHASE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->seqs.find(seq_id);
  if (it == s->seqs.end() || it->second.busy || !it->second.V) return CHASE_EINVAL;
  *V = it->second.V;
  *ldv = it->second.cfg.n;
  return CHASE_OK;
}

int chase_server_info(chase_server* s, int64_t* grouped_launches, int64_t* grouped_products,
                      size_t* bytes_in_use) {
  if (!s) return CHASE_EINVAL;
  int64_t launches = 0, products = 0;
  for (auto& b : s->batchers) {
    int64_t l = 0, p = 0;
    b->counters(&l, &p);
    launches += l;
    products += p;
  }
  if (grouped_launches) *grouped_launches = launches;
  if (grouped_products) *grouped_products = products;
  std::lock_guard<std::mutex> lk(s->mu);
  if (bytes_in_use) *bytes_in_use = s->used;
  return CHASE_OK;
}

int chase_server_end_sequence(chase_server* s, uint64_t seq_id) {
  if (!s) return CHASE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->seqs.find(seq_id);
  if (it == s->seqs.end()) return CHASE_EINVAL;
  if (it->second.busy) return CHASE_EBUSY;
  for (uint64_t t : s->queue)
    if (s->reqs[t].seq == seq_id) return CHASE_EBUSY;
  if (it->second.V) {
    (void)hipSetDevice(s->device);
    (void)hipFree(it->second.V);
  }
  s->used -= it->second.state_bytes;
  s->seqs.erase(it);
  s->cv.notify_all();
  return CHASE_OK;
}

const char* chase_server_last_error(chase_server* s) {
  return s ? s->last_error.c_str() : "NULL server";
}

void chase_server_destroy(chase_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& b : s->batchers) b.reset();
  (void)hipSetDevice(s->device);
  for (auto& kv : s->seqs)
    if (kv.second.V) (void)hipFree(kv.second.V);
  delete s;
}

}  // extern "C"
