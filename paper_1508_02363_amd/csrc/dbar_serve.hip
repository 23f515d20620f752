// Serving: a request queue with continuous batching for CGO solves (one k, one Q, one grid per request).
//
// Requests are grouped in classes by grid (N, L, M).  Each class owns a device workspace with `cap` slots, a HIP
// stream and a worker thread, so classes of different N run concurrently as different kernel shapes.  A worker
// repeats: admit queued requests into free slots (right-hand side, x = 0, first residual), run one lockstep Krylov
// cycle over every slot in flight, update the solutions and recompute the FP64 residuals, then finish the requests
// that converged (m = h(S), copy out) and free their slots.  New requests therefore join at the next cycle
// boundary while others are mid-solve.
//
// Admission is by device-memory footprint against the session budget.  A class reserves cap request footprints when
// it is created (cap = max_slots, or what the budget has left).  A request whose class does not exist and whose
// footprint the remaining budget cannot hold waits in the session's pending queue (first in, first out; later
// requests queue behind it, so none of them starves); a class that runs idle while requests are pending releases its
// workspace and its reservation, and the pending requests' classes are created as the budget allows.  Only a request
// larger than the whole budget is rejected.
//
// The paper motivates this by the need for solutions at many k (Section 1, and the outlook's parallelisation over
// k); each slot is an independent solve of the Section 4 system with Q -> q_k.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "dbar.h"
#include "dbar_launch.h"
#include "dbar_solver.h"

namespace dbar {

using Clock = std::chrono::steady_clock;

// Pinned host blocks, recycled per size: a request's potential is staged in one (so its upload is a DMA from pinned
// memory) and its results land in another (S, m and the GMRES record, copied from the device without blocking the
// worker's next cycle); dbar_poll copies the results out and returns both blocks.
struct PinnedPool {
  std::mutex mu;
  std::map<size_t, std::vector<void*>> free_blocks;
  void* get(size_t bytes) {
    {
      std::lock_guard<std::mutex> lock(mu);
      auto& v = free_blocks[bytes];
      if (!v.empty()) {
        void* p = v.back();
        v.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(mu);
    free_blocks[bytes].push_back(p);
  }
  ~PinnedPool() {
    for (auto& kv : free_blocks)
      for (void* p : kv.second) (void)hipHostFree(p);
  }
};

struct SReq {
  uint64_t ticket = 0;
  dbar_grid grid{};
  double k[2] = {0, 0};
  double tol = 1e-10;
  PinnedPool* pool = nullptr;
  c64* Q = nullptr;     // pinned: the potential (N*N)
  void* res = nullptr;  // pinned: S (N*N), m (N*N), then the GMRES record
  dbar_info info{};
  std::string err_msg;  // why the request ended with an error status
  int state = 0;  // 0 queued, 1 in flight, 2 done
  int iters = 0;
  size_t footprint = 0;
  Clock::time_point t_submit, t_done;
  size_t n() const { return (size_t)grid.n * grid.n; }
  size_t q_bytes() const { return n() * sizeof(c64); }
  size_t res_bytes() const { return 2 * n() * sizeof(c64) + sizeof(Ctl); }
  ~SReq() {
    if (pool) {
      pool->put(Q, q_bytes());
      pool->put(res, res_bytes());
    }
  }
};

// Results of finished slots on their way to the host: the copies run on the class's copy stream while the next cycle
// computes; the slots are admitted to again once `done` has completed.
struct Draining {
  hipEvent_t done = nullptr;
  std::vector<int> slots;
};

struct SClass {
  int N = 0, M = 11;
  double L = 1.0;
  int cap = 0;
  int prec = DBAR_MIXED;
  int restart = 20;
  size_t footprint = 0;
  Work w;
  Pipeline P;
  // the class's own twiddles (P points at these, not at the library's cache, which dbar_release() may free while
  // the session runs)
  Twiddles tw;
  hipStream_t stream = nullptr;
  std::vector<std::shared_ptr<SReq>> slots;
  std::deque<std::shared_ptr<SReq>> queue;
  std::thread th;
  DevBuf newmask, tolv;
  std::vector<int> h_new, h_live;
  std::vector<double> h_tol;
  std::vector<c64> h_k;  // per-slot k (host source of the async upload; stable until the stream synchronises)
  hipStream_t copy_stream = nullptr;  // result copies (device to pinned host), overlapping the next cycle
  hipEvent_t ev_results = nullptr;    // recorded on `stream` after a cycle: the finished slots' results are final
  std::deque<Draining> draining;
  bool ready = false;
  int error = 0;
  bool finished = false;  // the worker has returned: its thread can be joined
};

}  // namespace dbar

struct dbar_session {
  // first member: destroyed last, after every request that returns its pinned blocks to it
  dbar::PinnedPool pool;
  dbar_session_opts o{};
  size_t budget = 0, allocated = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<std::tuple<int, int, double>, std::unique_ptr<dbar::SClass>> classes;  // classes taking requests
  std::vector<std::unique_ptr<dbar::SClass>> retired;  // released classes (their workers exit; joined later)
  std::deque<std::shared_ptr<dbar::SReq>> pending;     // waiting for budget to create their class (FIFO)
  std::unordered_map<uint64_t, std::shared_ptr<dbar::SReq>> reqs;
  uint64_t next_ticket = 1;
  dbar_session_stats st{};
  std::atomic<bool> stop{false};
};

namespace dbar {

static size_t footprint_of(int N, int prec, int restart, int cap_hint) {
  const size_t n = (size_t)N * N;
  const bool mixed = prec == DBAR_MIXED;
  size_t per = n * ((size_t)(restart + 1) * (mixed ? sizeof(c32) : sizeof(c64)));  // Krylov basis
  per += n * sizeof(c64) * (mixed ? 7 : 6);                                       // x, b, T64, Q64, S, m (+ r64)
  per += mixed ? n * sizeof(c32) * 2 : 0;                                          // T32, Q32
  per += 2 * (size_t)N * sizeof(c64) + sizeof(Ctl) + 2 * kNMom * sizeof(c64);
  per += (size_t)2 * kNMom * 1024 * sizeof(double) + (size_t)(kMaxRestart + 3) * vec_blocks(n) * sizeof(double);
  (void)cap_hint;
  return per;
}

// Set up the class workspace (in the worker thread).
static int class_init(SClass& c) {
  int rc = c.w.setup(c.N, c.cap, c.restart, c.prec, false);
  if (rc) return rc;
  dbar_grid g{c.N, c.M, c.L};
  if ((rc = make_pipeline(&g, c.w, &c.P))) return rc;
  {
    std::vector<c64> h64(c.N);
    std::vector<c32> h32(c.N);
    host_twiddles(c.N, h64.data(), h32.data());
    if ((rc = c.tw.d64.ensure(c.N * sizeof(c64))) || (rc = c.tw.d32.ensure(c.N * sizeof(c32)))) return rc;
    if (hipMemcpy(c.tw.d64.p, h64.data(), c.N * sizeof(c64), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.tw.d32.p, h32.data(), c.N * sizeof(c32), hipMemcpyHostToDevice) != hipSuccess)
      return fail(DBAR_EDEVICE, "twiddle upload failed");
    c.P.tw64 = c.tw.d64.p;
    c.P.tw32 = c.tw.d32.p;
  }
  // GMRES on s = F^{-1} S; S and m come out of the residual evaluations
  c.P.xspace = true;
  const size_t nb = (size_t)c.cap * c.N * c.N * sizeof(c64);
  if ((rc = c.w.Sx.ensure(nb)) || (rc = c.w.mx.ensure(nb))) return rc;
  if ((rc = c.newmask.ensure(c.cap * sizeof(int)))) return rc;
  if ((rc = c.tolv.ensure(c.cap * sizeof(double)))) return rc;
  if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c.copy_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c.ev_results, hipEventDisableTiming) != hipSuccess)
    return fail(DBAR_EDEVICE, "stream creation failed");
  c.slots.assign(c.cap, nullptr);
  c.h_new.assign(c.cap, 0);
  c.h_live.assign(c.cap, 0);
  c.h_tol.assign(c.cap, 1e-10);
  c.h_k.assign(c.cap, c64{0.0, 0.0});
  c.w.B = c.cap;
  if (hipMemsetAsync(c.w.live.p, 0, c.cap * sizeof(int), c.stream) != hipSuccess ||
      hipMemsetAsync(c.w.act.p, 0, 3 * c.cap * sizeof(int), c.stream) != hipSuccess)
    return fail(DBAR_EDEVICE, "memset failed");
  return hipStreamSynchronize(c.stream) == hipSuccess ? DBAR_OK : fail(DBAR_EDEVICE, "sync failed");
}

static void schedule_pending(dbar_session* s);

// Take class c out of the session (under s->mu): requests for its grid now go to the pending queue or a new class.
static void detach_class(dbar_session* s, SClass& c) {
  for (auto it = s->classes.begin(); it != s->classes.end(); ++it)
    if (it->second.get() == &c) {
      s->retired.push_back(std::move(it->second));
      s->classes.erase(it);
      return;
    }
}

// The worker of a detached class: free its device memory, then return its reservation to the budget and admit what
// the pending queue can now hold.
static void destroy_streams(SClass& c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (c.copy_stream) (void)hipStreamSynchronize(c.copy_stream);
  for (auto& d : c.draining)
    if (d.done) (void)hipEventDestroy(d.done);
  c.draining.clear();
  if (c.ev_results) (void)hipEventDestroy(c.ev_results);
  if (c.stream) (void)hipStreamDestroy(c.stream);
  if (c.copy_stream) (void)hipStreamDestroy(c.copy_stream);
  c.ev_results = nullptr;
  c.stream = c.copy_stream = nullptr;
}

static void release_class(dbar_session* s, SClass& c) {
  destroy_streams(c);
  c.w = Work();
  c.tw = Twiddles();
  c.newmask = DevBuf();
  c.tolv = DevBuf();
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->allocated -= (size_t)c.cap * c.footprint;
    s->st.bytes_reserved = s->allocated;
    s->st.classes_released += 1;
    c.finished = true;
    schedule_pending(s);
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
}

// Hand slot b's request back (under s->mu): its info from the GMRES record in its result block (status: the
// convergence set at the cycle end, or `err`), the slot free for admission.
static void finish_slot(dbar_session* s, SClass& c, int b, int err, const char* why = "") {
  auto r = c.slots[b];
  if (err != DBAR_OK) r->err_msg = why;
  if (err == DBAR_OK && r->res) {
    const c64* S = static_cast<const c64*>(r->res);
    Ctl cc;
    std::memcpy(&cc, S + 2 * r->n(), sizeof(Ctl));
    r->info.iters = cc.iters;
    r->info.outer = cc.cycles;
    r->info.rel_residual = cc.bnorm > 0.0 ? cc.rnorm / cc.bnorm : 0.0;
    r->info.cond_estimate = cc.kappa;
    r->info.err_estimate = cc.kappa * r->info.rel_residual;
    r->info.m1_re = -S[0].im;  // m1 = i S(0)
    r->info.m1_im = S[0].re;
  } else {
    r->info.status = err == DBAR_OK ? DBAR_EDEVICE : err;
  }
  r->state = 2;
  r->t_done = Clock::now();
  c.slots[b] = nullptr;
  s->st.in_flight -= 1;
  s->st.completed += 1;
  s->st.bytes_in_use -= r->footprint;
}

// Requests whose result copies have completed, oldest first (wait: block until all have).
static void complete_copies(dbar_session* s, SClass& c, bool wait) {
  bool any = false;
  while (!c.draining.empty()) {
    Draining& d = c.draining.front();
    const hipError_t e = wait ? hipEventSynchronize(d.done) : hipEventQuery(d.done);
    if (e == hipErrorNotReady) break;
    {
      std::lock_guard<std::mutex> lock(s->mu);
      for (int b : d.slots)
        finish_slot(s, c, b, e == hipSuccess ? DBAR_OK : DBAR_EDEVICE,
                    e == hipSuccess ? "" : "the copy of the results to the host failed");
    }
    (void)hipEventDestroy(d.done);
    c.draining.pop_front();
    any = true;
  }
  if (any) s->cv_done.notify_all();
}

static void worker(dbar_session* s, SClass* cp) {
  SClass& c = *cp;
  (void)hipSetDevice(s->device);
  int rc = class_init(c);
  {
    std::lock_guard<std::mutex> lock(s->mu);
    c.ready = rc == DBAR_OK;
    c.error = rc;
    if (rc) {  // the requests routed to this class end with the error; the class gives its reservation back
      for (auto& r : c.queue) {
        r->state = 2;
        r->info.status = rc;
        r->err_msg = "the serving worker for this grid could not set up: " + g_last_error;
        r->t_done = Clock::now();
        s->st.queued -= 1;
      }
      c.queue.clear();
      detach_class(s, c);
    }
  }
  if (rc) {
    release_class(s, c);
    return;
  }
  Work& w = c.w;
  const size_t n = w.n;
  const bool mixed = c.prec == DBAR_MIXED;
  const size_t V_bs = n * (w.m + 1);
  BatchCfg cfg;
  cfg.tol = 1e-10;
  cfg.max_iter = 1000;
  cfg.reorth = 1;
  cfg.check_every = 4;
  cfg.inner_tol = 1e-6;  // x-space inner solves
  cfg.orth_window = kDefaultOrthWindow;
  // direct launches: a stream capture in one worker thread makes calls of the other workers (pinned allocations,
  // event queries, copies) fail with "not permitted when stream is capturing"
  cfg.use_graph = 0;
  bool retire = false;
  while (!s->stop.load()) {
    complete_copies(s, c, false);
    // ---- admission at the cycle boundary
    std::vector<int> admitted;
    bool any_live = false;
    {
      std::unique_lock<std::mutex> lock(s->mu);
      for (int b = 0; b < c.cap; ++b) any_live |= c.slots[b] != nullptr;  // in flight or draining
      if (!any_live && c.queue.empty()) {
        if (!s->pending.empty()) {  // idle while others wait for budget: release this class
          detach_class(s, c);
          retire = true;
          break;
        }
        s->cv_work.wait_for(lock, std::chrono::milliseconds(2));
        continue;
      }
      for (int b = 0; b < c.cap && !c.queue.empty(); ++b) {
        if (c.slots[b]) continue;
        auto r = c.queue.front();
        c.queue.pop_front();
        r->state = 1;
        c.slots[b] = r;
        admitted.push_back(b);
        s->st.queued -= 1;
        s->st.in_flight += 1;
        s->st.bytes_in_use += r->footprint;
      }
    }
    if (!admitted.empty()) {
      std::fill(c.h_new.begin(), c.h_new.end(), 0);
      for (int b : admitted) {
        SReq& r = *c.slots[b];
        c.h_new[b] = 1;
        c.h_live[b] = 1;
        w.full_host[b] = 0;  // the slot's new solve starts with the Gram-Schmidt window (its device flag: the check)
        c.h_tol[b] = r.tol;
        (void)hipMemcpyAsync(static_cast<c64*>(w.Q64.p) + (size_t)b * n, r.Q, n * sizeof(c64), hipMemcpyHostToDevice,
                             c.stream);
        c.h_k[b] = c64{r.k[0], r.k[1]};
        (void)hipMemcpyAsync(static_cast<c64*>(w.kvals.p) + b, &c.h_k[b], sizeof(c64), hipMemcpyHostToDevice,
                             c.stream);
        launch_phase_tables(static_cast<const c64*>(w.kvals.p) + b, c.N, c.L, static_cast<c64*>(w.ex.p) + (size_t)b * c.N,
                            static_cast<c64*>(w.ey.p) + (size_t)b * c.N, static_cast<c32*>(w.ex32.p) + (size_t)b * c.N,
                            static_cast<c32*>(w.ey32.p) + (size_t)b * c.N, 1, c.stream);
        (void)hipMemsetAsync(static_cast<c64*>(w.x.p) + (size_t)b * n, 0, n * sizeof(c64), c.stream);
        // host sources (request Q, per-slot tables, masks) stay untouched until the stream synchronises below
      }
      const int* nm = static_cast<const int*>(c.newmask.p);
      (void)hipMemcpyAsync(c.newmask.p, c.h_new.data(), c.cap * sizeof(int), hipMemcpyHostToDevice, c.stream);
      (void)hipMemcpyAsync(w.live.p, c.h_live.data(), c.cap * sizeof(int), hipMemcpyHostToDevice, c.stream);
      (void)hipMemcpyAsync(c.tolv.p, c.h_tol.data(), c.cap * sizeof(double), hipMemcpyHostToDevice, c.stream);
      if (mixed) launch_convert<float, double>(w.Q64.p, n, w.Q32.p, n, n, c.cap, nm, 1.0, c.stream);
      c.P.rhs_x(w.Q64.p, n, w.V.p, V_bs, mixed, c.cap, nm, 0u, c.stream);  // the first basis vector
      launch_reduce(static_cast<double*>(w.part_vec.p), 1, c.P.rhs_blocks(),
                    static_cast<double*>(w.nred.p), c.cap, nm, c.stream);
      launch_ctl_check(w, 0.0, 1, nm, static_cast<const double*>(c.tolv.p), c.stream);
      launch_zero_done(w, nm, false, c.stream);  // admitted requests with b = 0: S = m = 0
    }
    bool computing = false;
    for (int b = 0; b < c.cap; ++b) computing |= c.h_live[b] != 0;
    if (!computing) {  // only slots whose results are still on their way to the host
      complete_copies(s, c, true);
      continue;
    }
    // ---- one Krylov cycle for everything in flight
    launch_ctl_start(w, mixed ? 0.3 : 0.5, mixed ? cfg.inner_tol : 0.0, static_cast<const double*>(c.tolv.p),
                     c.stream);
    int ran;
    if (mixed) {
      ran = krylov_cycle<float>(c.P, w, cfg, c.restart, c.stream);
      end_cycle<float>(c.P, w, ran, w.r64.p, c.stream);
    } else {
      ran = krylov_cycle<double>(c.P, w, cfg, c.restart, c.stream);
      end_cycle<double>(c.P, w, ran, w.V.p, c.stream);
    }
    launch_ctl_check(w, 0.0, 0, nullptr, static_cast<const double*>(c.tolv.p), c.stream);
    // (x-space: the residual evaluation wrote the next cycle's FP32 basis vector itself)
    std::vector<int> live_now(c.cap);
    (void)hipMemcpyAsync(live_now.data(), w.live.p, c.cap * sizeof(int), hipMemcpyDeviceToHost, c.stream);
    if (hipStreamSynchronize(c.stream) != hipSuccess) {
      std::lock_guard<std::mutex> lock(s->mu);
      c.error = DBAR_EDEVICE;
      for (auto& r : c.slots)
        if (r) {
          r->state = 2;
          r->info.status = DBAR_EDEVICE;
          r->err_msg = std::string("the serving worker's stream failed: ") + hipGetErrorString(hipGetLastError());
          r->t_done = Clock::now();
        }
      s->cv_done.notify_all();
      return;
    }
    // ---- finish converged (or exhausted) requests
    std::vector<int> fin;
    for (int b = 0; b < c.cap; ++b) {
      if (!c.slots[b] || !c.h_live[b]) continue;
      c.slots[b]->iters += ran;
      const bool done = live_now[b] == 0;
      const bool exhausted = !done && c.slots[b]->iters >= cfg.max_iter;
      if (done || exhausted || ran == 0) {
        c.h_live[b] = 0;
        fin.push_back(b);
        c.slots[b]->info.status = done ? DBAR_OK : DBAR_ENOCONV;
      }
    }
    if (fin.empty()) continue;
    (void)hipMemcpyAsync(w.live.p, c.h_live.data(), c.cap * sizeof(int), hipMemcpyHostToDevice, c.stream);
    // the finished slots' S, m (the last residual evaluation's) and GMRES records go to pinned blocks on the copy
    // stream; the next cycle does not write them (the slots are not live) and starts at once
    Draining d;
    d.slots = fin;
    bool ok = hipEventRecord(c.ev_results, c.stream) == hipSuccess &&
              hipStreamWaitEvent(c.copy_stream, c.ev_results, 0) == hipSuccess &&
              hipEventCreateWithFlags(&d.done, hipEventDisableTiming) == hipSuccess;
    int err = DBAR_EDEVICE;
    const char* why = "queueing the result copies failed";
    for (size_t i = 0; i < fin.size() && ok; ++i) {
      const int b = fin[i];
      SReq& r = *c.slots[b];
      r.res = s->pool.get(r.res_bytes());
      if (!r.res) {
        ok = false;
        err = DBAR_ENOMEM;
        why = "pinned host memory for the results could not be allocated";
        break;
      }
      c64* S = static_cast<c64*>(r.res);
      ok = hipMemcpyAsync(S, static_cast<c64*>(w.Sx.p) + (size_t)b * n, n * sizeof(c64), hipMemcpyDeviceToHost,
                          c.copy_stream) == hipSuccess &&
           hipMemcpyAsync(S + n, static_cast<c64*>(w.mx.p) + (size_t)b * n, n * sizeof(c64), hipMemcpyDeviceToHost,
                          c.copy_stream) == hipSuccess &&
           hipMemcpyAsync(S + 2 * n, static_cast<Ctl*>(w.ctl.p) + b, sizeof(Ctl), hipMemcpyDeviceToHost,
                          c.copy_stream) == hipSuccess;
    }
    ok = ok && hipEventRecord(d.done, c.copy_stream) == hipSuccess;
    if (!ok) {  // no pinned memory or a runtime error: these requests end with an error
      (void)hipStreamSynchronize(c.copy_stream);
      if (d.done) (void)hipEventDestroy(d.done);
      std::lock_guard<std::mutex> lock(s->mu);
      for (int b : fin) finish_slot(s, c, b, err, why);
      s->cv_done.notify_all();
      continue;
    }
    c.draining.push_back(d);
  }
  complete_copies(s, c, true);
  if (retire) release_class(s, c);
}

// Create the class of request r if the remaining budget holds at least one of its footprints (under s->mu); null
// if it does not, or (with *failed set) if the class's worker thread could not be started.
static SClass* create_class(dbar_session* s, const SReq& r, bool* failed) {
  const size_t fp = r.footprint;
  const size_t left = s->budget > s->allocated ? s->budget - s->allocated : 0;
  const int cap = (int)std::min<size_t>((size_t)s->o.max_slots, left / fp);
  if (cap < 1) return nullptr;
  // join the workers of released classes that have returned (not the calling worker itself, which releases its class
  // and admits pending requests before it returns)
  for (auto it = s->retired.begin(); it != s->retired.end();) {
    if ((*it)->finished && (*it)->th.get_id() != std::this_thread::get_id()) {
      if ((*it)->th.joinable()) (*it)->th.join();
      it = s->retired.erase(it);
    } else {
      ++it;
    }
  }
  auto c = std::make_unique<SClass>();
  c->N = r.grid.n;
  c->M = r.grid.M;
  c->L = r.grid.L;
  c->cap = cap;
  c->prec = s->o.precision;
  c->restart = s->o.restart;
  c->footprint = fp;
  SClass* cp = c.get();
  // (the worker touches only its class until it takes s->mu, which the caller holds until the class is inserted)
  try {
    cp->th = std::thread(worker, s, cp);
  } catch (...) {
    *failed = true;
    return nullptr;
  }
  s->allocated += (size_t)cap * fp;
  s->st.bytes_reserved = s->allocated;
  s->st.classes_created += 1;
  s->classes.emplace(std::make_tuple(r.grid.n, r.grid.M, r.grid.L), std::move(c));
  return cp;
}

// Move pending requests, oldest first, into their classes (creating classes as the budget allows); stop at the first
// request whose class cannot be created yet (under s->mu).
static void schedule_pending(dbar_session* s) {
  if (s->stop.load()) return;
  while (!s->pending.empty()) {
    auto r = s->pending.front();
    auto it = s->classes.find(std::make_tuple(r->grid.n, r->grid.M, r->grid.L));
    bool failed = false;
    SClass* c = it != s->classes.end() ? it->second.get() : create_class(s, *r, &failed);
    if (failed) {  // no worker for its grid: the request ends with an error rather than waiting for ever
      s->pending.pop_front();
      r->state = 2;
      r->info.status = DBAR_EDEVICE;
      r->err_msg = "the serving worker thread for this grid could not be started";
      r->t_done = Clock::now();
      s->st.queued -= 1;
      s->cv_done.notify_all();
      continue;
    }
    if (!c) break;
    c->queue.push_back(r);
    s->pending.pop_front();
  }
  s->cv_work.notify_all();
}

}  // namespace dbar

using namespace dbar;

extern "C" {

size_t dbar_request_footprint(const dbar_grid* grid, int32_t precision, int32_t restart) {
  if (validate_grid(grid)) return 0;
  if (restart <= 0) restart = precision == DBAR_FP64 ? 40 : 20;
  return footprint_of(grid->n, precision, restart, 1);
}

int dbar_session_create(const dbar_session_opts* opts, dbar_session** out) {
  if (!out) return fail(DBAR_EINVAL, "out is NULL");
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt < 1) {
    (void)hipGetLastError();
    return fail(DBAR_EDEVICE, "no HIP device available");
  }
  auto* s = new dbar_session();
  if (opts) s->o = *opts;
  if (s->o.max_slots <= 0) s->o.max_slots = 64;
  if (s->o.precision != DBAR_FP64) s->o.precision = DBAR_MIXED;
  if (s->o.restart <= 0) s->o.restart = s->o.precision == DBAR_MIXED ? 20 : 40;
  if (s->o.restart > kMaxRestart) s->o.restart = kMaxRestart;
  (void)hipGetDevice(&s->device);
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  s->budget = s->o.hbm_budget_bytes ? s->o.hbm_budget_bytes : (size_t)(0.8 * (double)fr);
  *out = s;
  return DBAR_OK;
}

int dbar_submit(dbar_session* s, const dbar_grid* grid, const double* Q, const double* k, double tol,
                uint64_t* ticket) {
  if (!s || !ticket || !Q || !k) return fail(DBAR_EINVAL, "NULL argument");
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DBAR_EINVAL, "tol must be finite and > 0");
  const size_t n = (size_t)grid->n * grid->n;
  for (size_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(Q[i])) return fail(DBAR_EINVAL, "Q contains NaN or Inf");
  if (!std::isfinite(k[0]) || !std::isfinite(k[1])) return fail(DBAR_EINVAL, "k contains NaN or Inf");
  auto r = std::make_shared<SReq>();
  r->grid = *grid;
  r->k[0] = k[0];
  r->k[1] = k[1];
  r->tol = tol;
  r->pool = &s->pool;
  r->Q = static_cast<c64*>(s->pool.get(r->q_bytes()));
  if (!r->Q) return fail(DBAR_ENOMEM, "pinned host memory for the request's potential could not be allocated");
  std::memcpy(r->Q, Q, n * sizeof(c64));
  r->footprint = footprint_of(grid->n, s->o.precision, s->o.restart, 1);
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lock(s->mu);
  if (r->footprint > s->budget) {
    s->st.rejected += 1;
    return fail(DBAR_ENOMEM, "request footprint (" + std::to_string(r->footprint) +
                                 " bytes) exceeds the session's HBM budget (" + std::to_string(s->budget) + " bytes)");
  }
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->st.submitted += 1;
  s->st.queued += 1;
  *ticket = r->ticket;
  // behind any request already waiting for budget; otherwise straight into its class
  s->pending.push_back(r);
  schedule_pending(s);
  return DBAR_OK;
}

// Copy a finished request's results out (outside the session lock: up to two N x N arrays) and report its status.
static int deliver(const std::shared_ptr<SReq>& r, double* S_out, double* m_out, dbar_info* info, double* latency_s) {
  const size_t n = r->n();
  if (r->res) {
    const c64* S = static_cast<const c64*>(r->res);
    if (S_out) std::memcpy(S_out, S, n * sizeof(c64));
    if (m_out) std::memcpy(m_out, S + n, n * sizeof(c64));
  }
  if (info) *info = r->info;
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  const int st = r->info.status;
  if (st == DBAR_OK || st == DBAR_ENOCONV) return st;
  return fail(st, !r->err_msg.empty() ? r->err_msg
                                      : std::string(st == DBAR_ENOMEM ? "the serving worker could not allocate its workspace"
                                                                      : "device failure in the serving worker"));
}

int dbar_poll(dbar_session* s, uint64_t ticket, double* S_out, double* m_out, dbar_info* info, double* latency_s) {
  if (!s) return fail(DBAR_EINVAL, "session is NULL");
  std::shared_ptr<SReq> r;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(DBAR_ENOTFOUND, "unknown ticket");
    if (it->second->state != 2) return DBAR_EAGAIN;
    r = it->second;
    s->reqs.erase(it);
  }
  return deliver(r, S_out, m_out, info, latency_s);
}

int dbar_wait(dbar_session* s, uint64_t ticket, double* S_out, double* m_out, dbar_info* info, double* latency_s) {
  if (!s) return fail(DBAR_EINVAL, "session is NULL");
  std::shared_ptr<SReq> r;
  {
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
      auto it = s->reqs.find(ticket);
      if (it == s->reqs.end()) return fail(DBAR_ENOTFOUND, "unknown ticket");
      if (it->second->state == 2) {
        r = it->second;
        s->reqs.erase(it);
        break;
      }
      s->cv_done.wait_for(lock, std::chrono::milliseconds(50));
    }
  }
  return deliver(r, S_out, m_out, info, latency_s);
}

int dbar_session_get_stats(dbar_session* s, dbar_session_stats* st) {
  if (!s || !st) return fail(DBAR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(s->mu);
  *st = s->st;
  return DBAR_OK;
}

void dbar_session_destroy(dbar_session* s) {
  if (!s) return;
  s->stop.store(true);
  s->cv_work.notify_all();
  // a worker may move its class from `classes` to `retired` while it exits: collect the threads under the lock, join
  // them outside it
  std::vector<SClass*> all;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    for (auto& kv : s->classes) all.push_back(kv.second.get());
    for (auto& c : s->retired) all.push_back(c.get());
  }
  for (SClass* c : all)
    if (c->th.joinable()) c->th.join();
  for (auto& kv : s->classes) destroy_streams(*kv.second);
  for (auto& c : s->retired) destroy_streams(*c);
  delete s;
}

}  // extern "C"
