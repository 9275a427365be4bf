// Serving loop: continuous batching of matrix-element requests of different
// processes, precisions and sizes on one GPU.
//
// The paper measured that several host processes feeding one GPU reach the
// throughput plateau at smaller grids and raise the combined throughput
// (section 2, Fig. 1); this is the same idea inside one process.  Requests
// are queued on submission.  A scheduler thread admits them onto free slots
// (one HIP stream each, default priority) as soon as a slot is free and the
// device workspace of all running requests stays within the HBM budget; the
// queue is scanned in arrival order and a request that does not fit is
// passed over by a later one that does (a request larger than the whole
// budget runs alone).  Admitted requests run concurrently on their streams;
// completion is signalled by a host function enqueued behind the request's
// kernels, which frees the slot and the budget and wakes the scheduler.
// Process constants and good-helicity lists stay resident in the processes;
// each request runs exactly the kernels a standalone call runs, so its result
// does not depend on what runs beside it.
//
// A test double can replace the device: it "completes" each request after
// fake_ns_per_event * nevt nanoseconds without touching the GPU, so the
// scheduler, admission and latency accounting can be tested on a CPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mgme.h"
#include "registry.h"

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
  int slot = -1;
  int status = MGME_OK;
  bool done = false;
  Clock::time_point t_submit, t_done;
};

}  // namespace

struct mgme_server {
  mgme_server_config cfg{};
  int device = 0;
  std::vector<hipStream_t> streams;
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
  long long submitted = 0, completed = 0, failed = 0, events = 0;
  std::vector<double> latencies_ms;
  bool any_submit = false;
  Clock::time_point first_submit, last_done;
  int running = 0, max_running = 0;
  long long peak_ws = 0;
};

extern "C" int mgme_process_info(const mgme_process* proc, mgme_info* out);

namespace {

thread_local std::string g_serr;

int sfail(int code, const char* msg) {
  g_serr = msg;
  return code;
}

// Called with s->mu held.
void finish_locked(mgme_server* s, int slot, int status) {
  Request* r = s->slot_req[slot];
  s->slot_req[slot] = nullptr;
  r->status = status;
  r->done = true;
  r->t_done = Clock::now();
  s->in_use -= r->footprint;
  s->running -= 1;
  if (status == MGME_OK) {
    s->completed += 1;
    s->events += r->nevt;
    s->latencies_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
  } else {
    s->failed += 1;
  }
  s->last_done = r->t_done;
  s->cv_sched.notify_all();
  s->cv_done.notify_all();
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

void scheduler_loop(mgme_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    int free_slot = -1;
    for (size_t i = 0; i < s->slot_req.size(); ++i)
      if (!s->slot_req[i]) {
        free_slot = (int)i;
        break;
      }
    Request* r = nullptr;
    if (free_slot >= 0 && !s->queue.empty()) {
      // find the first queued request that fits
      for (size_t i = 0; i < s->queue.size(); ++i) {
        Request* c = s->queue[i];
        if (s->running == 0 || s->in_use + c->footprint <= s->cfg.hbm_budget_bytes) {
          r = c;
          s->queue.erase(s->queue.begin() + (long)i);
          break;
        }
      }
    }
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
    s->peak_ws = std::max(s->peak_ws, s->in_use);
    if (s->cfg.fake_executor) {
      const auto due = Clock::now() + std::chrono::nanoseconds((long long)(s->cfg.fake_ns_per_event * r->nevt));
      s->fake_due.emplace(due, free_slot);
      s->cv_timer.notify_all();
      continue;
    }
    lk.unlock();
    int rc = mgme_matrix_element(r->proc, r->mom, r->nevt, r->ld, r->prec, r->out, s->streams[free_slot]);
    if (rc == MGME_OK) {
      HostCb* cb = new (std::nothrow) HostCb{s, free_slot};
      if (!cb || hipLaunchHostFunc(s->streams[free_slot], on_complete, cb) != hipSuccess) {
        delete cb;
        // fall back to waiting for the stream from this thread
        const hipError_t e = hipStreamSynchronize(s->streams[free_slot]);
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
    finish_locked(s, slot, MGME_OK);
  }
}

}  // namespace

extern "C" {

const char* mgme_server_last_error(void) { return g_serr.c_str(); }

int mgme_server_create(const mgme_server_config* cfg, int device, mgme_server** out) {
  if (!cfg || !out) return sfail(MGME_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 64 || cfg->hbm_budget_bytes < 0)
    return sfail(MGME_EINVAL, "n_slots must be 1..64 and the budget non-negative");
  if (cfg->fake_executor && !(cfg->fake_ns_per_event >= 0.0)) return sfail(MGME_EINVAL, "bad fake duration");
  mgme_server* s = new (std::nothrow) mgme_server();
  if (!s) return sfail(MGME_ENOMEM, "host allocation");
  s->cfg = *cfg;
  s->device = device;
  s->slot_req.assign(cfg->n_slots, nullptr);
  if (!cfg->fake_executor) {
    if (hipSetDevice(device) != hipSuccess) {
      delete s;
      return sfail(MGME_EDEVICE, "hipSetDevice");
    }
    // keep freed workspace in the stream-ordered pool up to the budget
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      unsigned long long thr = (unsigned long long)cfg->hbm_budget_bytes;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    for (int i = 0; i < cfg->n_slots; ++i) {
      hipStream_t st;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        delete s;
        return sfail(MGME_EDEVICE, "hipStreamCreate");
      }
      s->streams.push_back(st);
    }
  }
  s->scheduler = std::thread(scheduler_loop, s);
  if (cfg->fake_executor) s->timer = std::thread(timer_loop, s);
  *out = s;
  return MGME_OK;
}

int mgme_server_submit(mgme_server* s, const mgme_process* proc, const double* d_mom, long long nevt, long long ld,
                       int precision, double* d_me, unsigned long long* id) {
  if (!s || !id || (!proc && !s->cfg.fake_executor)) return sfail(MGME_EINVAL, "NULL argument");
  if (nevt < 1 || ld < nevt || (!s->cfg.fake_executor && (!d_mom || !d_me)))
    return sfail(MGME_EINVAL, "bad batch");
  if (precision < MGME_FP64 || precision > MGME_FP64_FP32COLOUR) return sfail(MGME_EINVAL, "unknown precision");
  long long ws = 0;
  if (s->cfg.fake_executor) ws = (long long)s->cfg.fake_bytes_per_event * nevt;
  else if (mgme_workspace_bytes(proc, nevt, precision, &ws) != MGME_OK) return sfail(MGME_EINVAL, "bad process");
  Request* r = new (std::nothrow) Request();
  if (!r) return sfail(MGME_ENOMEM, "host allocation");
  r->proc = proc;
  r->mom = d_mom;
  r->nevt = nevt;
  r->ld = ld;
  r->prec = precision;
  r->out = d_me;
  r->footprint = ws;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) {
    delete r;
    return sfail(MGME_EINVAL, "server is stopping");
  }
  r->id = s->next_id++;
  s->requests[r->id] = r;
  s->queue.push_back(r);
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
  delete r;
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
  out->peak_workspace_bytes = s->peak_ws;
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
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto& kv : s->requests) delete kv.second;
  delete s;
  return MGME_OK;
}

}  // extern "C"
