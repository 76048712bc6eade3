// snn_server.cpp -- serving simulation requests on one GPU with continuous
// admission by device-memory budget (the C ABI's snn_server_* calls).
//
// A request is a defined, not yet built network and a number of steps.
// Requests wait in one queue in submission order.  `slots` worker threads
// take them: a free worker takes the first queued request whose known memory
// need fits what the budget has left, builds it, simulates it on the
// network's own stream and releases its device memory the moment it is done
// (snn_release: the raster and counters stay on the host), which admits the
// next request.  So requests submitted while others run start as soon as a
// slot and memory are free, and the slots' networks run on the device at the
// same time.  The budget is exact: every device allocation of a served
// network passes through the server, which refuses one that would exceed
// the budget; the build then fails and releases what it had, and the request
// goes back to the head of the queue with that amount as its known need.  A
// request that cannot fit even with nothing else on the device fails with
// SNN_E_BUDGET.  Each network is advanced by the same kernels it would run
// alone, so its result does not depend on the others.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/snn.h"
#include "snn_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Job;

}  // namespace

struct snn_server {
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> queue;                                  // submission order
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;  // until the result is taken
  size_t in_use = 0, peak = 0;                             // device bytes granted to served networks
  uint32_t running = 0;
  uint64_t next_ticket = 1, done = 0, failed = 0;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

struct Job {
  snn_server* srv = nullptr;
  uint64_t ticket = 0;
  snn_net* net = nullptr;
  uint64_t steps = 0;
  snn_device orig{};
  bool orig_have = false;
  int32_t state = SNN_JOB_QUEUED;
  snn_status status = SNN_OK;
  std::string err;
  size_t bytes = 0, bytes_peak = 0;  // device bytes held now, and at most
  size_t need = 0;                   // known need: bytes held when an allocation was refused, plus that allocation
  bool refused = false;
  int attempts = 0;
  std::unordered_map<void*, size_t> sizes;
  double t_submit = 0, t_start = 0, t_done = 0;
};

// Device memory of a served network: granted only within the budget.
void* srv_alloc(size_t bytes, void* user) {
  Job* j = static_cast<Job*>(user);
  snn_server* s = j->srv;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->in_use + bytes > s->budget) {
      j->refused = true;
      j->need = j->bytes + bytes;
      return nullptr;
    }
    s->in_use += bytes;
    s->peak = std::max(s->peak, s->in_use);
    j->bytes += bytes;
    j->bytes_peak = std::max(j->bytes_peak, j->bytes);
  }
  void* p = nullptr;
  if (j->orig_have && j->orig.alloc) {
    p = j->orig.alloc(bytes, j->orig.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!p) {
    s->in_use -= bytes;
    j->bytes -= bytes;
  } else {
    j->sizes[p] = bytes;
  }
  return p;
}

void srv_free(void* p, void* user) {
  Job* j = static_cast<Job*>(user);
  snn_server* s = j->srv;
  if (j->orig_have && j->orig.free) j->orig.free(p, j->orig.user);
  else (void)hipFree(p);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = j->sizes.find(p);
  if (it != j->sizes.end()) {
    s->in_use -= it->second;
    j->bytes -= it->second;
    j->sizes.erase(it);
  }
  s->cv.notify_all();  // memory returned: a waiting request may fit now
}

// First queued job whose known need fits the memory left (with the lock held).
Job* pick(snn_server* s) {
  const size_t left = s->budget - s->in_use;
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
    if ((*it)->need <= left) {
      Job* j = *it;
      s->queue.erase(it);
      return j;
    }
  return nullptr;
}

void finish(snn_server* s, Job* j, snn_status st, const char* msg) {
  // with the lock held
  j->status = st;
  if (st != SNN_OK) j->err = msg ? msg : "";
  j->state = st == SNN_OK ? SNN_JOB_DONE : SNN_JOB_FAILED;
  j->t_done = now_s();
  if (st == SNN_OK) ++s->done;
  else ++s->failed;
  s->cv.notify_all();
}

void worker(snn_server* s) {
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || (j = pick(s)) != nullptr; });
      if (s->stop && !j) return;
      j->state = SNN_JOB_RUNNING;
      if (!j->attempts++) j->t_start = now_s();
      ++s->running;
    }
    (void)hipSetDevice(snn::net_device(j->net));
    j->refused = false;
    snn_status st = snn_build(j->net);
    if (st == SNN_E_NOMEM && j->refused) {
      // the budget refused an allocation; the failed build has released its memory
      std::lock_guard<std::mutex> lk(s->mu);
      --s->running;
      if (j->need > s->budget || (s->running == 0 && s->in_use == 0)) {
        finish(s, j, SNN_E_BUDGET, "the network needs more device memory than the whole budget");
      } else {
        j->state = SNN_JOB_QUEUED;  // back to the head: it goes first once its need fits
        s->queue.push_front(j);
        s->cv.notify_all();
      }
      continue;
    }
    std::string msg;
    if (st == SNN_OK) st = snn_simulate_steps(j->net, j->steps);
    if (st != SNN_OK) msg = snn_last_error(j->net);
    const snn_status rs = snn_release(j->net);  // the raster and counters stay; the memory goes back now
    if (st == SNN_OK && rs != SNN_OK && rs != SNN_E_STATE) {
      st = rs;
      msg = snn_last_error(j->net);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    --s->running;
    finish(s, j, st, msg.c_str());
  }
}

}  // namespace

extern "C" {

snn_status snn_server_create(size_t hbm_budget, uint32_t slots, snn_server** out) {
  if (!out || hbm_budget == 0 || slots == 0 || slots > 64) return SNN_E_INVALID;
  *out = nullptr;
  snn_server* s = new (std::nothrow) snn_server();
  if (!s) return SNN_E_NOMEM;
  s->budget = hbm_budget;
  try {
    for (uint32_t k = 0; k < slots; ++k) s->workers.emplace_back(worker, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
    return SNN_E_NOMEM;
  }
  *out = s;
  return SNN_OK;
}

void snn_server_destroy(snn_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Job* j : s->queue) finish(s, j, SNN_E_STATE, "server destroyed before the request ran");
    s->queue.clear();
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  // results never taken: the networks (released, or never built) go back to
  // the caller, who still holds their handles, with their own allocators
  for (auto& kv : s->jobs) snn::net_set_allocator(kv.second->net, kv.second->orig, kv.second->orig_have);
  delete s;
}

snn_status snn_server_submit(snn_server* s, snn_net* net, uint64_t steps, uint64_t* ticket) {
  if (!s || !net || !ticket) return SNN_E_INVALID;
  if (!snn::net_is_fresh(net)) return SNN_E_STATE;
  // a lower bound of its need: the 4-byte synapse words alone
  if (4 * snn::net_planned_synapses(net) > s->budget) return SNN_E_BUDGET;
  auto j = std::make_unique<Job>();
  j->srv = s;
  j->net = net;
  j->steps = steps;
  snn::net_allocator(net, &j->orig, &j->orig_have);
  snn_device d = j->orig;
  d.alloc = srv_alloc;
  d.free = srv_free;
  d.user = j.get();
  snn::net_set_allocator(net, d, true);
  j->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return SNN_E_STATE;
  j->ticket = s->next_ticket++;
  *ticket = j->ticket;
  s->queue.push_back(j.get());
  s->jobs[j->ticket] = std::move(j);
  s->cv.notify_all();
  return SNN_OK;
}

snn_status snn_server_poll(snn_server* s, uint64_t ticket, int32_t* state) {
  if (!s || !state) return SNN_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return SNN_E_INVALID;
  *state = it->second->state;
  return SNN_OK;
}

snn_status snn_server_wait(snn_server* s, uint64_t ticket, double timeout_s) {
  if (!s) return SNN_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return SNN_E_INVALID;
  Job* j = it->second.get();
  auto ended = [&] { return j->state == SNN_JOB_DONE || j->state == SNN_JOB_FAILED; };
  if (timeout_s < 0) s->cv.wait(lk, ended);
  else if (!s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ended)) return SNN_E_STATE;
  return SNN_OK;
}

snn_status snn_server_result(snn_server* s, uint64_t ticket, snn_net** net, snn_job_info* info) {
  if (!s || !net) return SNN_E_INVALID;
  std::unique_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return SNN_E_INVALID;
    if (it->second->state != SNN_JOB_DONE && it->second->state != SNN_JOB_FAILED) return SNN_E_STATE;
    j = std::move(it->second);
    s->jobs.erase(it);
  }
  snn::net_set_allocator(j->net, j->orig, j->orig_have);
  *net = j->net;
  if (info) {
    info->status = j->status;
    info->attempts = (uint32_t)j->attempts;
    info->t_submit = j->t_submit;
    info->t_start = j->t_start;
    info->t_done = j->t_done;
    info->device_bytes_peak = j->bytes_peak;
    snprintf(info->error, sizeof info->error, "%s", j->err.c_str());
  }
  return j->status;
}

snn_status snn_server_get_stats(snn_server* s, snn_server_stats* out) {
  if (!s || !out) return SNN_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  out->budget = s->budget;
  out->in_use = s->in_use;
  out->peak = s->peak;
  out->queued = (uint32_t)s->queue.size();
  out->running = s->running;
  out->done = s->done;
  out->failed = s->failed;
  return SNN_OK;
}

}  // extern "C"
