// Serving loop: continuous batching of matrix-element requests of different
// processes, precisions and sizes on one GPU.
//
// The paper measured that several host processes feeding one GPU reach the
// throughput plateau at smaller grids and raise the combined throughput
// (section 2, Fig. 1); this is the same idea inside one process.  Requests
// are queued on submission.  A scheduler thread admits them onto free slots
// (one HIP stream each, default priority) as soon as a slot is free and the
// HBM footprint of all running requests (momenta, results and staging
// workspace) stays within the budget.  The queue is scanned in arrival order
// and a request that does not fit may be passed over by a later one that
// does, but only a bounded number of times: once a request has been passed
// over max_pass_over times, nothing behind it is admitted until it fits.  A
// request whose footprint exceeds the whole budget is split into parts that
// fit (an event's |M|^2 does not depend on the batch it is computed in).
// Admitted requests run concurrently on their streams; completion is
// signalled by a host function enqueued behind the request's kernels, which
// frees the slot and the budget and wakes the scheduler.  Process constants
// and good-helicity lists stay resident in the processes; each request runs
// exactly the kernels of a standalone call, so its result does not depend on
// what runs beside it.
//
// With use_graphs, a request's launches are captured into a HIP graph on its
// slot's stream and replayed; the staging workspace then belongs to the slot
// (allocated once, outside any graph), and an instantiated graph is kept per
// (slot, process, precision, power-of-two batch size) and updated in place
// for the next request of that kind.
//
// A test double can replace the device: it "completes" each request after
// fake_ns_per_event * nevt nanoseconds without touching the GPU, so the
// scheduler, admission, splitting, failure handling and latency accounting
// can be tested on a CPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/mgme.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  unsigned long long id = 0;
  const mgme_process* proc = nullptr;
  const double* mom = nullptr;
  long long nevt = 0, ld = 0;
  int prec = 0;
  double* out = nullptr;
  long long footprint = 0;
  int passed = 0;             // times a later request was admitted ahead of this one
  hipEvent_t ready = nullptr; // recorded on the submitter's stream (owned by the parent)
  Request* parent = nullptr;  // set on the parts of a split request
  int parts_left = 0;         // parent of a split request: parts not yet finished
  int slot = -1;
  int status = MGME_OK;
  bool done = false;
  Clock::time_point t_submit, t_done;
};

using GraphKey = std::tuple<const mgme_process*, int, int>;  // process, precision, log2 bucket

}  // namespace

struct mgme_server {
  mgme_server_config cfg{};
  int device = 0;
  long long budget = 0;
  std::vector<hipStream_t> streams;
  std::vector<void*> slot_ws;
  std::vector<std::map<GraphKey, hipGraphExec_t>> graphs;  // per slot
  std::vector<Request*> slot_req;
  long long in_use = 0;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<unsigned long long, Request*> requests;
  unsigned long long next_id = 1;
  bool stopping = false;
  std::thread scheduler;
  // test double
  std::thread timer;
  std::multimap<Clock::time_point, int> fake_due;  // completion time -> slot
  std::condition_variable cv_timer;
  // statistics
  long long submitted = 0, completed = 0, failed = 0, events = 0, split = 0;
  long long graph_launches = 0, graph_instantiations = 0;
  std::vector<double> latencies_ms;
  bool any_submit = false;
  Clock::time_point first_submit, last_done;
  int running = 0, max_running = 0;
  long long peak_in_use = 0;
};

namespace {

thread_local std::string g_serr;

int sfail(int code, const char* msg) {
  g_serr = msg;
  return code;
}

constexpr long long kDefaultSlotWorkspace = 1ll << 30;
constexpr int kDefaultMaxPassOver = 4;

// Completes a user-visible request (a whole request, or the parent of a
// split one).  Called with s->mu held, possibly from a host function enqueued
// on a stream, so it makes no HIP call (the readiness event is released when
// the request is waited for).
void complete_locked(mgme_server* s, Request* r, int status, Clock::time_point t) {
  r->status = status;
  r->done = true;
  r->t_done = t;
  if (status == MGME_OK) {
    s->completed += 1;
    s->events += r->nevt;
    s->latencies_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
  } else {
    s->failed += 1;
  }
  s->last_done = t;
  s->cv_done.notify_all();
}

// The request on `slot` finished with `status`.  Called with s->mu held.
void finish_locked(mgme_server* s, int slot, int status) {
  Request* r = s->slot_req[slot];
  s->slot_req[slot] = nullptr;
  s->in_use -= r->footprint;
  s->running -= 1;
  const auto t = Clock::now();
  if (r->parent) {
    Request* p = r->parent;
    if (status != MGME_OK && p->status == MGME_OK) p->status = status;
    delete r;
    if (--p->parts_left == 0) complete_locked(s, p, p->status, t);
  } else {
    complete_locked(s, r, status, t);
  }
  s->cv_sched.notify_all();
}

struct HostCb {
  mgme_server* s;
  int slot;
};

void on_complete(void* p) {
  HostCb* cb = static_cast<HostCb*>(p);
  {
    std::lock_guard<std::mutex> lk(cb->s->mu);
    finish_locked(cb->s, cb->slot, MGME_OK);
  }
  delete cb;
}

int log2_bucket(long long n) {
  int b = 0;
  while ((1ll << b) < n) ++b;
  return b;
}

// Captures the request's launches on the slot's stream and replays them as a
// graph, updating the slot's instantiated graph of the same kind in place.
// Runs on the scheduler thread without the lock; only this thread touches the
// slot's graphs, and a slot holds one request at a time, so no instance is
// updated while it runs.
int launch_graph(mgme_server* s, int slot, const Request* r) {
  hipStream_t st = s->streams[slot];
  const mgme::Workspace ws{s->slot_ws[slot], s->cfg.slot_workspace_bytes};
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return mgme::set_error(MGME_EDEVICE, "hipStreamBeginCapture");
  const int rc = mgme::matrix_element_ws(r->proc, r->mom, r->nevt, r->ld, r->prec, r->out, &ws, st);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  if (rc != MGME_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != MGME_OK ? rc : mgme::set_error(MGME_EDEVICE, "hipStreamEndCapture");
  }
  hipGraphExec_t& ex = s->graphs[slot][GraphKey{r->proc, r->prec, log2_bucket(r->nevt)}];
  if (ex) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(ex, g, &err_node, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(ex);
      ex = nullptr;
    }
  }
  if (!ex) {
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      ex = nullptr;
      (void)hipGraphDestroy(g);
      return mgme::set_error(MGME_EDEVICE, "hipGraphInstantiate");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->graph_instantiations += 1;
  }
  (void)hipGraphDestroy(g);
  e = hipGraphLaunch(ex, st);
  if (e != hipSuccess) return mgme::set_error(MGME_EDEVICE, "hipGraphLaunch");
  std::lock_guard<std::mutex> lk(s->mu);
  s->graph_launches += 1;
  return MGME_OK;
}

// Admission: the first queued request, in arrival order, that fits beside the
// running ones; a request passed over max_pass_over times stops the scan, so
// that nothing behind it is admitted until it fits.  Called with s->mu held.
Request* admit_locked(mgme_server* s) {
  const int max_pass = s->cfg.max_pass_over > 0 ? s->cfg.max_pass_over : kDefaultMaxPassOver;
  for (size_t i = 0; i < s->queue.size(); ++i) {
    Request* c = s->queue[i];
    if (s->running == 0 || s->in_use + c->footprint <= s->budget) {
      for (size_t j = 0; j < i; ++j) s->queue[j]->passed += 1;
      s->queue.erase(s->queue.begin() + (long)i);
      return c;
    }
    if (c->passed >= max_pass) break;
  }
  return nullptr;
}

void scheduler_loop(mgme_server* s) {
  if (!s->cfg.fake_executor) (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    int free_slot = -1;
    for (size_t i = 0; i < s->slot_req.size(); ++i)
      if (!s->slot_req[i]) {
        free_slot = (int)i;
        break;
      }
    Request* r = (free_slot >= 0 && !s->queue.empty()) ? admit_locked(s) : nullptr;
    if (!r) {
      if (s->stopping && s->queue.empty() && s->running == 0) return;
      s->cv_sched.wait(lk);
      continue;
    }
    r->slot = free_slot;
    s->slot_req[free_slot] = r;
    s->in_use += r->footprint;
    s->running += 1;
    s->max_running = std::max(s->max_running, s->running);
    s->peak_in_use = std::max(s->peak_in_use, s->in_use);
    if (s->cfg.fake_executor) {
      const auto due = Clock::now() + std::chrono::nanoseconds((long long)(s->cfg.fake_ns_per_event * r->nevt));
      s->fake_due.emplace(due, free_slot);
      s->cv_timer.notify_all();
      continue;
    }
    const hipEvent_t ready = r->parent ? r->parent->ready : r->ready;
    lk.unlock();
    hipStream_t st = s->streams[free_slot];
    int rc = MGME_OK;
    if (ready && hipStreamWaitEvent(st, ready, 0) != hipSuccess) rc = mgme::set_error(MGME_EDEVICE, "hipStreamWaitEvent");
    if (rc == MGME_OK) {
      rc = s->cfg.use_graphs ? launch_graph(s, free_slot, r)
                             : mgme_matrix_element(r->proc, r->mom, r->nevt, r->ld, r->prec, r->out, st);
    }
    if (rc == MGME_OK) {
      HostCb* cb = new (std::nothrow) HostCb{s, free_slot};
      if (!cb || hipLaunchHostFunc(st, on_complete, cb) != hipSuccess) {
        delete cb;
        // fall back to waiting for the stream from this thread
        const hipError_t e = hipStreamSynchronize(st);
        lk.lock();
        finish_locked(s, free_slot, e == hipSuccess ? MGME_OK : MGME_EDEVICE);
        continue;
      }
      lk.lock();
    } else {
      lk.lock();
      finish_locked(s, free_slot, rc);
    }
  }
}

void timer_loop(mgme_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->fake_due.empty()) {
      if (s->stopping && s->queue.empty() && s->running == 0) return;
      s->cv_timer.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    const auto due = s->fake_due.begin()->first;
    if (Clock::now() < due) {
      s->cv_timer.wait_until(lk, due);
      continue;
    }
    const int slot = s->fake_due.begin()->second;
    s->fake_due.erase(s->fake_due.begin());
    const Request* r = s->slot_req[slot];
    const bool fail = s->cfg.fake_fail_nevt > 0 && r->nevt == s->cfg.fake_fail_nevt;
    finish_locked(s, slot, fail ? MGME_EDEVICE : MGME_OK);
  }
}

// HBM footprint of `n` events of a request: momenta and results, plus the
// staging workspace unless that belongs to the slots.
long long footprint(const mgme_server* s, const mgme_process* proc, long long n, int prec) {
  if (s->cfg.fake_executor) return s->cfg.fake_bytes_per_event * n;
  long long ws = 0;
  if (!s->cfg.use_graphs) (void)mgme_workspace_bytes(proc, n, prec, &ws);
  return n * (32ll * mgme::process_n_ext(proc) + 8) + ws;
}

void destroy_device_state(mgme_server* s) {
  for (auto& m : s->graphs)
    for (auto& kv : m)
      if (kv.second) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  s->streams.clear();
  for (void* p : s->slot_ws)
    if (p) (void)hipFree(p);
  s->slot_ws.clear();
}

}  // namespace

extern "C" {

const char* mgme_server_last_error(void) { return g_serr.c_str(); }

int mgme_server_create(const mgme_server_config* cfg, int device, mgme_server** out) {
  if (!cfg || !out) return sfail(MGME_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 64 || cfg->hbm_budget_bytes < 0 || cfg->slot_workspace_bytes < 0 ||
      cfg->max_pass_over < 0)
    return sfail(MGME_EINVAL, "n_slots must be 1..64 and the budget, slot workspace and pass-over bound non-negative");
  if (cfg->fake_executor && !(cfg->fake_ns_per_event >= 0.0 && cfg->fake_bytes_per_event >= 0))
    return sfail(MGME_EINVAL, "bad fake duration or footprint");
  mgme_server* s = new (std::nothrow) mgme_server();
  if (!s) return sfail(MGME_ENOMEM, "host allocation");
  s->cfg = *cfg;
  s->device = device;
  s->slot_req.assign(cfg->n_slots, nullptr);
  if (cfg->fake_executor) {
    s->budget = cfg->hbm_budget_bytes > 0 ? cfg->hbm_budget_bytes : LLONG_MAX;
  } else {
    if (hipSetDevice(device) != hipSuccess) {
      delete s;
      return sfail(MGME_EDEVICE, "hipSetDevice");
    }
    if (cfg->use_graphs && s->cfg.slot_workspace_bytes == 0) s->cfg.slot_workspace_bytes = kDefaultSlotWorkspace;
    for (int i = 0; i < cfg->n_slots; ++i) {
      hipStream_t st;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        destroy_device_state(s);
        delete s;
        return sfail(MGME_EDEVICE, "hipStreamCreate");
      }
      s->streams.push_back(st);
      if (cfg->use_graphs) {
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)s->cfg.slot_workspace_bytes) != hipSuccess) {
          (void)hipGetLastError();
          destroy_device_state(s);
          delete s;
          return sfail(MGME_ENOMEM, "slot workspace");
        }
        s->slot_ws.push_back(p);
      }
    }
    s->graphs.resize(cfg->n_slots);
    if (cfg->hbm_budget_bytes > 0) {
      s->budget = cfg->hbm_budget_bytes;
    } else {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        destroy_device_state(s);
        delete s;
        return sfail(MGME_EDEVICE, "hipMemGetInfo");
      }
      s->budget = (long long)(0.8 * (double)free_b);
    }
    // keep freed workspace in the stream-ordered pool up to the budget
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      unsigned long long thr = (unsigned long long)s->budget;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  }
  s->scheduler = std::thread(scheduler_loop, s);
  if (cfg->fake_executor) s->timer = std::thread(timer_loop, s);
  *out = s;
  return MGME_OK;
}

int mgme_server_submit(mgme_server* s, const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                       int precision, double* d_me, void* hip_stream, unsigned long long* id) {
  if (!s || !id || (!proc && !s->cfg.fake_executor)) return sfail(MGME_EINVAL, "NULL argument");
  if (nevt < 1 || ld < nevt || (!s->cfg.fake_executor && (!d_mom || !d_me)))
    return sfail(MGME_EINVAL, "bad batch");
  if (precision < MGME_FP64 || precision > MGME_FP64_FP32COLOUR) return sfail(MGME_EINVAL, "unknown precision");
  if (!s->cfg.fake_executor && s->cfg.use_graphs &&
      mgme::workspace_min_bytes(proc, precision) > s->cfg.slot_workspace_bytes)
    return sfail(MGME_EINVAL, "slot workspace smaller than one 64-event sub-batch of this process");
  // parts of at most `part` events each fit the budget (a whole request if it does)
  long long part = nevt;
  while (part > 64 && footprint(s, proc, part, precision) > s->budget) part = (part / 2 + 63) / 64 * 64;
  std::vector<Request*> parts;
  Request* r = new (std::nothrow) Request();
  if (!r) return sfail(MGME_ENOMEM, "host allocation");
  r->proc = proc;
  r->mom = d_mom;
  r->nevt = nevt;
  r->ld = ld;
  r->prec = precision;
  r->out = d_me;
  r->footprint = footprint(s, proc, nevt, precision);
  r->t_submit = Clock::now();
  if (part < nevt) {
    for (long long start = 0; start < nevt; start += part) {
      Request* q = new (std::nothrow) Request();
      if (!q) {
        for (Request* x : parts) delete x;
        delete r;
        return sfail(MGME_ENOMEM, "host allocation");
      }
      q->proc = proc;
      q->nevt = std::min(part, nevt - start);
      q->mom = d_mom ? d_mom + start : nullptr;
      q->ld = ld;
      q->prec = precision;
      q->out = d_me ? d_me + start : nullptr;
      q->footprint = footprint(s, proc, q->nevt, precision);
      q->parent = r;
      q->t_submit = r->t_submit;
      parts.push_back(q);
    }
    r->parts_left = (int)parts.size();
  }
  if (!s->cfg.fake_executor) {
    // the request's launches wait for what the submitter enqueued before
    if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r->ready, (hipStream_t)hip_stream) != hipSuccess) {
      (void)hipGetLastError();
      if (r->ready) (void)hipEventDestroy(r->ready);
      for (Request* x : parts) delete x;
      delete r;
      return sfail(MGME_EDEVICE, "recording the readiness event");
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    for (Request* x : parts) delete x;
    delete r;
    return sfail(MGME_EINVAL, "server is stopping");
  }
  r->id = s->next_id++;
  s->requests[r->id] = r;
  if (parts.empty()) {
    s->queue.push_back(r);
  } else {
    for (Request* q : parts) s->queue.push_back(q);
    s->split += 1;
  }
  s->submitted += 1;
  if (!s->any_submit) {
    s->any_submit = true;
    s->first_submit = r->t_submit;
  }
  *id = r->id;
  s->cv_sched.notify_all();
  return MGME_OK;
}

int mgme_server_wait(mgme_server* s, unsigned long long id, double* latency_ms) {
  if (!s) return sfail(MGME_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(id);
  if (it == s->requests.end()) return sfail(MGME_EINVAL, "unknown request");
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  const int st = r->status;
  s->requests.erase(it);
  if (r->ready) (void)hipEventDestroy(r->ready);
  delete r;
  if (st != MGME_OK) g_serr = "request failed on the device";
  return st;
}

int mgme_server_drain(mgme_server* s) {
  if (!s) return sfail(MGME_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
  return MGME_OK;
}

int mgme_server_get_stats(mgme_server* s, mgme_server_stats* out) {
  if (!s || !out) return sfail(MGME_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->events = s->events;
  std::vector<double> v = s->latencies_ms;
  std::sort(v.begin(), v.end());
  auto q = [&](double f) {
    if (v.empty()) return 0.0;
    const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(f * (double)v.size()) - 1);
    return v[k];
  };
  out->p50_ms = q(0.50);
  out->p99_ms = q(0.99);
  double sum = 0.0;
  for (double x : v) sum += x;
  out->mean_ms = v.empty() ? 0.0 : sum / (double)v.size();
  out->max_ms = v.empty() ? 0.0 : v.back();
  out->wall_s = s->any_submit && s->completed + s->failed > 0
                    ? std::chrono::duration<double>(s->last_done - s->first_submit).count()
                    : 0.0;
  out->max_concurrent = s->max_running;
  out->peak_footprint_bytes = s->peak_in_use;
  out->budget_bytes = s->budget == LLONG_MAX ? 0 : s->budget;
  out->split_requests = s->split;
  out->graph_launches = s->graph_launches;
  out->graph_instantiations = s->graph_instantiations;
  return MGME_OK;
}

int mgme_server_destroy(mgme_server* s) {
  if (!s) return MGME_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_sched.notify_all();
    s->cv_timer.notify_all();
  }
  s->scheduler.join();
  if (s->timer.joinable()) s->timer.join();
  destroy_device_state(s);
  for (auto& kv : s->requests) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  delete s;
  return MGME_OK;
}

}  // extern "C"
