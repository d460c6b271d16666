// Serving loop: continuous batching of top-k requests over device-resident
// arrays.
//
// Clients submit requests (device pointers, as for topk_select_batched) from
// any thread.  One dispatcher thread per server:
//   * completes launches whose event has fired (latency = completion seen on
//     the host - arrival), releasing their HBM footprint; a launch whose
//     kernels raised an internal check flag (drtopk_check on its stream)
//     fails all of its requests with DRTOPK_EDEVICE;
//   * when a launch stream is free, takes the oldest queued request: one too
//     large for a workgroup (n > 2^22 or k > 2048) runs alone through the
//     single-problem path; otherwise the queued small requests are admitted in
//     arrival order while the in-flight footprint stays within the budget and
//     launched as one batched call on that stream;
//   * otherwise polls the busy streams, or sleeps until a request arrives.
// Requests that arrive while batches run join the next launch on another
// stream, so their work overlaps on the device with the running batches.
// The `plain` mode launches one request at a time through topk_select /
// kth_select: the per-request loop the batched server is measured against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "drtopk.h"

namespace {

using Clock = std::chrono::steady_clock;

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

struct Req {
  drtopk_problem_t p{};
  uint64_t fp = 0;
  bool large = false;  // runs alone through the single-problem path
  Clock::time_point arrival{};
  double latency_us = 0;
  int status = DRTOPK_OK;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<uint64_t> items;  // tickets in flight on this stream
  uint64_t bytes = 0;
  bool busy = false;
};

}  // namespace

struct drtopk_server {
  drtopk_server_config_t cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> reqs;        // requests not yet reported by a drain: ticket base + i is reqs[i]
  uint64_t base = 0;           // ticket of reqs.front(); earlier tickets were reported by a drain
  std::deque<uint64_t> qsmall, qlarge;  // submitted, not yet admitted, in arrival order
  std::vector<Slot> slots;
  uint64_t inflight_bytes = 0, max_inflight_bytes = 0;
  uint64_t launches = 0, launched_items = 0;
  std::vector<double> lat;  // completed latencies since the last stats reset
  bool stop = false;
  bool broken = false;      // the dispatcher failed (out of host memory): requests fail
  std::thread th;

  Req& at(uint64_t t) { return reqs[t - base]; }
  bool queued() const { return !qsmall.empty() || !qlarge.empty(); }
  void loop();
  void run();
  void fail_all();
  bool complete_ready();
};

// The dispatcher, with a failure path: if it cannot allocate, it waits for
// the launches in flight and completes every unfinished request with
// DRTOPK_ENOMEM, so no waiter blocks forever; later submits fail.
void drtopk_server::run() {
  try {
    loop();
  } catch (...) {
    fail_all();
  }
}

void drtopk_server::fail_all() {
  for (auto& sl : slots) (void)hipStreamSynchronize(sl.stream);
  std::lock_guard<std::mutex> g(mu);
  broken = true;
  for (auto& r : reqs)
    if (!r.done) {
      r.status = DRTOPK_ENOMEM;
      r.done = true;
    }
  qsmall.clear();
  qlarge.clear();
  for (auto& sl : slots) {
    sl.items.clear();
    sl.busy = false;
  }
  cv_done.notify_all();
}

// Marks finished launches complete; returns true if any slot is still busy.
bool drtopk_server::complete_ready() {
  bool busy = false;
  for (auto& sl : slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) {
      busy = true;
      continue;
    }
    const Clock::time_point now = Clock::now();
    // the launch has finished: a failed internal check of any of its kernels
    // fails every request of the launch
    uint32_t flags = 0;
    const bool flagged = q == hipSuccess && drtopk_check(sl.stream, &flags) != DRTOPK_OK;
    std::lock_guard<std::mutex> g(mu);
    for (uint64_t t : sl.items) {
      Req& r = at(t);
      r.latency_us = us_between(r.arrival, now);
      if ((q != hipSuccess || flagged) && r.status == DRTOPK_OK) r.status = DRTOPK_EDEVICE;
      r.done = true;
      lat.push_back(r.latency_us);
    }
    if (q != hipSuccess) (void)hipGetLastError();
    inflight_bytes -= sl.bytes;
    sl.bytes = 0;
    sl.items.clear();
    sl.busy = false;
    cv_done.notify_all();
  }
  return busy;
}

void drtopk_server::loop() {
  (void)hipSetDevice(device);
  std::vector<drtopk_problem_t> batch;
  for (;;) {
    const bool busy = complete_ready();
    Slot* free_slot = nullptr;
    for (auto& sl : slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    std::vector<uint64_t> take;
    uint64_t bytes = 0;
    {
      std::unique_lock<std::mutex> g(mu);
      if (stop && !queued() && !busy) return;
      if (free_slot && queued()) {
        // the oldest request decides: a large one runs alone, else a batch of small ones
        const bool large_first = !qlarge.empty() && (qsmall.empty() || qlarge.front() < qsmall.front());
        std::deque<uint64_t>& q = large_first ? qlarge : qsmall;
        const uint32_t cap = large_first ? 1u : cfg.max_batch;
        while (!q.empty() && take.size() < cap) {
          Req& r = at(q.front());
          // admission by footprint; a request larger than the budget runs alone
          if (inflight_bytes + bytes + r.fp > cfg.hbm_budget && (inflight_bytes + bytes) > 0) break;
          bytes += r.fp;
          take.push_back(q.front());
          q.pop_front();
        }
        if (!take.empty()) {
          inflight_bytes += bytes;
          max_inflight_bytes = std::max(max_inflight_bytes, inflight_bytes);
        }
      }
      if (take.empty()) {
        if (!busy) {
          cv_work.wait(g, [&] { return stop || queued(); });
          continue;
        }
      }
    }
    if (take.empty()) {  // streams busy: poll again (sleeping would add the timer's slack to latency)
      std::this_thread::yield();
      continue;
    }
    batch.clear();
    {
      std::lock_guard<std::mutex> g(mu);
      for (uint64_t t : take) batch.push_back(at(t).p);
    }
    int st = DRTOPK_OK;
    std::vector<int> each(take.size(), DRTOPK_OK);
    if (cfg.plain || take.size() == 1) {  // one request: the single-problem path directly
      for (size_t i = 0; i < batch.size(); ++i) {
        const drtopk_problem_t& p = batch[i];
        each[i] = p.out_vals ? topk_select(p.keys, p.n, p.k, (int)p.dtype, p.out_vals, p.out_idx, free_slot->stream)
                             : kth_select(p.keys, p.n, p.k, (int)p.dtype, p.out_kth, free_slot->stream);
        if (each[i] == DRTOPK_OK && p.out_vals && p.out_kth &&
            hipMemcpyAsync(p.out_kth, static_cast<char*>(p.out_vals) + 4ull * (p.k - 1), 4, hipMemcpyDeviceToDevice,
                           free_slot->stream) != hipSuccess)
          each[i] = DRTOPK_EDEVICE;
      }
    } else {
      st = topk_select_batched(batch.data(), (uint32_t)batch.size(), free_slot->stream);
      std::fill(each.begin(), each.end(), st);
    }
    if (hipEventRecord(free_slot->ev, free_slot->stream) != hipSuccess) {
      (void)hipGetLastError();
      std::fill(each.begin(), each.end(), (int)DRTOPK_EDEVICE);
    }
    {
      std::lock_guard<std::mutex> g(mu);
      ++launches;
      launched_items += take.size();
      for (size_t i = 0; i < take.size(); ++i) at(take[i]).status = each[i];
      free_slot->items = take;
      free_slot->bytes = bytes;
      free_slot->busy = true;
    }
  }
}

extern "C" {

int drtopk_server_create(const drtopk_server_config_t* cfg, drtopk_server_t** out) {
  if (!cfg || !out) return DRTOPK_EINVAL;
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->streams < 1 || cfg->streams > 16 || cfg->plain > 1) return DRTOPK_EINVAL;
  drtopk_server* s = new (std::nothrow) drtopk_server();
  if (!s) return DRTOPK_ENOMEM;
  s->cfg = *cfg;
  if (s->cfg.hbm_budget == 0) s->cfg.hbm_budget = 8ull << 30;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return DRTOPK_EDEVICE;
  }
  s->slots.resize(cfg->streams);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      for (auto& x : s->slots) {
        if (x.ev) (void)hipEventDestroy(x.ev);
        if (x.stream) (void)hipStreamDestroy(x.stream);
      }
      delete s;
      return DRTOPK_EDEVICE;
    }
  }
  try {
    s->th = std::thread([s] { s->run(); });
  } catch (...) {
    for (auto& x : s->slots) {
      (void)hipEventDestroy(x.ev);
      (void)hipStreamDestroy(x.stream);
    }
    delete s;
    return DRTOPK_ENOMEM;
  }
  *out = s;
  return DRTOPK_OK;
}

}  // extern "C"

namespace {

int submit_at(drtopk_server_t* s, const drtopk_problem_t* req, Clock::time_point arrival, uint64_t* ticket) {
  if (!s || !req || !ticket) return DRTOPK_EINVAL;
  if (!req->out_vals && !req->out_kth) return DRTOPK_EINVAL;
  uint64_t fp = 0;
  int st = drtopk_footprint(req->n, req->k, (int)req->dtype, &fp);
  if (st) return st;
  if (!req->keys) return DRTOPK_EINVAL;
  int32_t route = 0, alpha = 0;
  st = drtopk_batched_alpha(req->n, req->k, &route, &alpha, nullptr);
  if (st) return st;
  Req r;
  r.p = *req;
  r.fp = fp;
  // 64-bit keys always take the single-problem path (the batched kernel is 32-bit)
  const int base = (int)(req->dtype & ~(uint32_t)DRTOPK_SMALLEST);
  r.large = route == 0 || base == DRTOPK_U64 || base == DRTOPK_I64 || base == DRTOPK_F64;
  r.arrival = arrival;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return DRTOPK_EINVAL;
    if (s->broken) return DRTOPK_ENOMEM;
    try {
      s->reqs.push_back(r);
      *ticket = s->base + s->reqs.size() - 1;
      (r.large ? s->qlarge : s->qsmall).push_back(*ticket);
    } catch (...) {
      return DRTOPK_ENOMEM;
    }
  }
  s->cv_work.notify_one();
  return DRTOPK_OK;
}

}  // namespace

extern "C" {

int drtopk_server_submit(drtopk_server_t* s, const drtopk_problem_t* req, uint64_t* ticket) {
  return submit_at(s, req, Clock::now(), ticket);
}

int drtopk_server_wait(drtopk_server_t* s, uint64_t ticket, double* latency_us) {
  if (!s) return DRTOPK_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  if (ticket < s->base || ticket >= s->base + s->reqs.size()) return DRTOPK_EINVAL;
  s->cv_done.wait(g, [&] { return s->at(ticket).done; });
  const Req& r = s->at(ticket);
  if (latency_us) *latency_us = r.latency_us;
  return r.status;
}

int drtopk_server_drain(drtopk_server_t* s) {
  if (!s) return DRTOPK_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  s->cv_done.wait(g, [&] {
    if (s->queued()) return false;
    for (const auto& sl : s->slots)
      if (sl.busy) return false;
    return true;
  });
  // nothing is queued or in flight: every record is complete; report and drop them
  int st = DRTOPK_OK;
  for (const Req& r : s->reqs)
    if (r.status != DRTOPK_OK) st = r.status;
  s->base += s->reqs.size();
  s->reqs.clear();
  return st;
}

int drtopk_server_stats(drtopk_server_t* s, drtopk_server_stats_t* out, int reset) {
  if (!s || !out) return DRTOPK_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof(*out));
  std::vector<double> v = s->lat;
  std::sort(v.begin(), v.end());
  out->completed = v.size();
  out->launches = s->launches;
  out->launched_items = s->launched_items;
  out->max_inflight_bytes = s->max_inflight_bytes;
  if (!v.empty()) {
    auto pct = [&](double q) {
      size_t i = (size_t)(q * (double)(v.size() - 1) + 0.5);
      return v[std::min(i, v.size() - 1)];
    };
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / (double)v.size();
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    out->max_us = v.back();
  }
  if (reset) {
    s->lat.clear();
    s->launches = 0;
    s->launched_items = 0;
    s->max_inflight_bytes = s->inflight_bytes;
  }
  return DRTOPK_OK;
}

int drtopk_server_replay(drtopk_server_t* s, const drtopk_problem_t* reqs, const double* arrival_us, uint32_t count,
                         double* latency_us, double* elapsed_us) {
  if (!s || (count && (!reqs || !arrival_us))) return DRTOPK_EINVAL;
  for (uint32_t i = 0; i < count; ++i) {
    uint64_t fp;
    if (i && arrival_us[i] < arrival_us[i - 1]) return DRTOPK_EINVAL;
    if ((!reqs[i].out_vals && !reqs[i].out_kth) || !reqs[i].keys) return DRTOPK_EINVAL;
    int st = drtopk_footprint(reqs[i].n, reqs[i].k, (int)reqs[i].dtype, &fp);
    if (st) return st;
  }
  std::vector<uint64_t> tickets(count);
  const Clock::time_point t0 = Clock::now();
  for (uint32_t i = 0; i < count; ++i) {
    const Clock::time_point due = t0 + std::chrono::duration_cast<Clock::duration>(
                                           std::chrono::duration<double, std::micro>(arrival_us[i]));
    while (Clock::now() < due) {
      if (due - Clock::now() > std::chrono::microseconds(50))
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    int st = submit_at(s, &reqs[i], due, &tickets[i]);  // latency counts from the scheduled arrival
    if (st) return st;
  }
  int st = DRTOPK_OK;
  for (uint32_t i = 0; i < count; ++i) {
    double l = 0;
    int e = drtopk_server_wait(s, tickets[i], &l);
    if (e) st = e;
    if (latency_us) latency_us[i] = l;
  }
  if (elapsed_us) *elapsed_us = us_between(t0, Clock::now());
  return st;
}

int drtopk_server_destroy(drtopk_server_t* s) {
  if (!s) return DRTOPK_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  int st = DRTOPK_OK;
  for (auto& sl : s->slots) {
    if (hipStreamSynchronize(sl.stream) != hipSuccess) st = DRTOPK_EDEVICE;
    (void)hipEventDestroy(sl.ev);
    (void)hipStreamDestroy(sl.stream);
  }
  delete s;
  return st;
}

}  // extern "C"
