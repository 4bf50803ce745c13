// Scheduling core of the HAVSampler serving loop: requests wait for a device slot within a
// memory budget, slots come in capacity classes of 2^k points, idle slots of other classes
// are released when the budget needs the room, and a worker thread runs continuous
// batching: every admitted request waiting for the device goes into the next batch, and up
// to one batch per flight (stream) is in flight at once. The core makes no device call
// itself. An executor does: it gives slots their memory, enqueues a batch, says when a
// batch has finished and hands back each request's result. The library instantiates the
// core with an executor over HIP; host-only tests instantiate it with one over the CPU
// oracle, so admission, queueing, rejection and routing are checked without a GPU.
//
// Executor requirements (E):
//   using SlotMem = ...;                    the executor's storage of one slot
//   size_t slot_bytes(int cls) const;       device bytes one slot of class cls holds
//   size_t fixed_bytes() const;             device bytes held for the server's life
//   int flights() const;                    batches that may be in flight at once (>= 1)
//   bool slot_alloc(Slot<SlotMem>& s);      give s (cls, n_cap and bytes set) its storage
//   void slot_free(Slot<SlotMem>& s);
//   hav_status_t launch(int f, const std::vector<Request<SlotMem>*>& reqs);
//       enqueue one batch on flight f and return at once: initialise every slot that is
//       not ready (and mark it ready), bring the clouds in, sample, bring the results back
//   int query(int f);                       1 finished, 0 still running, -1 failed
//   void drain(int f);                      wait until flight f is idle (after a failed launch)
//   void collect(Request<SlotMem>& r);      r.info, r.status and r.result from its slot
//   void on_worker_start();                 first call on the worker thread
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/hav.h"

namespace hav_serve {

constexpr int kMinClass = 12;  // 4,096 points
constexpr int kMaxClass = 24;  // 16,777,216 points

inline int class_of(int64_t n) {
  int k = kMinClass;
  while ((int64_t(1) << k) < n) ++k;
  return k;
}

template <class SlotMem>
struct Slot {
  int cls = 0;
  int64_t n_cap = 0;
  size_t bytes = 0;    // device bytes held
  bool ready = false;  // workspace initialised
  bool busy = false;
  SlotMem mem{};
};

template <class SlotMem>
struct Request {
  uint64_t ticket = 0;
  const float* xyz_host = nullptr;
  int64_t n = 0, m = 0;
  std::chrono::steady_clock::time_point t_submit, t_done;
  bool done = false;
  hav_status_t status = HAV_OK;
  Slot<SlotMem>* slot = nullptr;
  std::vector<int32_t> result;
  hav_info_t info{};
};

template <class E>
class Server {
 public:
  using SlotT = Slot<typename E::SlotMem>;
  using RequestT = Request<typename E::SlotMem>;

  Server(E exec, size_t budget, int32_t max_batch)
      : exec_(std::move(exec)), budget_(budget), max_batch_(max_batch) {
    flights_.resize(static_cast<size_t>(exec_.flights()));
    used_ = exec_.fixed_bytes();
  }
  Server(const Server&) = delete;
  Server& operator=(const Server&) = delete;
  ~Server() { shutdown(); }

  E& exec() { return exec_; }

  void start() { worker_ = std::thread([this] { worker_loop(); }); }

  // HAV_ERR_OUT_OF_MEMORY when one slot of the request's class cannot fit the budget
  // next to the memory the server holds for its life.
  hav_status_t submit(const float* xyz_host, int64_t N, int64_t M, uint64_t* ticket) {
    if (!xyz_host || !ticket || N < 1 || M < 1 || M > N || N > (int64_t(1) << kMaxClass))
      return HAV_ERR_INVALID_ARG;
    if (exec_.slot_bytes(class_of(N)) + exec_.fixed_bytes() > budget_) return HAV_ERR_OUT_OF_MEMORY;
    auto r = std::make_unique<RequestT>();
    r->xyz_host = xyz_host;
    r->n = N;
    r->m = M;
    r->t_submit = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> lk(mu_);
      r->ticket = next_ticket_++;
      *ticket = r->ticket;
      pending_.push_back(r.get());
      reqs_.emplace(r->ticket, std::move(r));
      ++stats_.submitted;
    }
    cv_.notify_one();
    return HAV_OK;
  }

  hav_status_t poll(uint64_t ticket, int32_t* idx_host, hav_info_t* info_host, double* latency_ms) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return HAV_ERR_INVALID_ARG;
    RequestT* r = it->second.get();
    if (!r->done) return HAV_NOT_READY;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    if (info_host) *info_host = r->info;
    if (idx_host && r->status == HAV_OK && !r->result.empty())
      std::memcpy(idx_host, r->result.data(), r->result.size() * sizeof(int32_t));
    const hav_status_t st = r->status;
    reqs_.erase(it);
    return st;
  }

  void stats(hav_server_stats_t* out) {
    std::lock_guard<std::mutex> lk(mu_);
    *out = stats_;
    out->hbm_used = used_;
    out->slots = static_cast<int64_t>(slots_.size());
  }

  // Finish the batches in flight, drop requests not yet admitted, free every slot.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_) return;
      stop_ = true;
      for (RequestT* r : pending_) r->done = true;  // (never admitted: dropped)
      pending_.clear();
    }
    cv_.notify_one();
    if (worker_.joinable()) worker_.join();
    for (auto& s : slots_) exec_.slot_free(*s);
    slots_.clear();
    stopped_ = true;
  }

 private:
  struct Flight {
    bool busy = false;
    std::vector<RequestT*> reqs;
  };

  // A free slot able to hold n points: the smallest class that fits, else a new one
  // within the budget (releasing idle slots, smallest first, if that makes room); when
  // no new slot fits, a free slot of a larger class. Caller holds the lock.
  SlotT* acquire_slot(int64_t n) {
    const int want = class_of(n);
    SlotT* best = nullptr;
    for (auto& s : slots_)
      if (!s->busy && s->cls >= want && (!best || s->cls < best->cls)) best = s.get();
    if (best && best->cls == want) {
      best->busy = true;
      return best;
    }
    const size_t need = exec_.slot_bytes(want);
    if (used_ + need > budget_) {
      std::vector<SlotT*> idle;
      size_t idle_bytes = 0;
      for (auto& s : slots_)
        if (!s->busy) {
          idle.push_back(s.get());
          idle_bytes += s->bytes;
        }
      if (used_ - idle_bytes + need > budget_) {
        if (best) {
          best->busy = true;
          return best;
        }
        return nullptr;
      }
      std::sort(idle.begin(), idle.end(), [](SlotT* a, SlotT* b) { return a->bytes < b->bytes; });
      best = nullptr;  // (it may be released below)
      for (SlotT* s : idle) {
        if (used_ + need <= budget_) break;
        used_ -= s->bytes;
        exec_.slot_free(*s);
        ++stats_.evictions;
        for (auto it = slots_.begin(); it != slots_.end(); ++it)
          if (it->get() == s) {
            slots_.erase(it);
            break;
          }
      }
    }
    auto s = std::make_unique<SlotT>();
    s->cls = want;
    s->n_cap = int64_t(1) << want;
    s->bytes = need;
    if (!exec_.slot_alloc(*s)) {
      if (best) {
        best->busy = true;
        return best;
      }
      return nullptr;
    }
    s->busy = true;
    used_ += need;
    ++stats_.slots_created;
    slots_.push_back(std::move(s));
    return slots_.back().get();
  }

  // Caller holds the lock.
  void finish_request(RequestT* r, hav_status_t st) {
    r->t_done = std::chrono::steady_clock::now();
    r->status = st;
    if (st == HAV_OK && r->slot) exec_.collect(*r);
    // A request that failed may leave its slot's workspace dirty (a wait that gave up
    // clears the workspace's validity mark; a launch sequence that failed part way can
    // leave claims in its tables): the slot is initialised again before its next request.
    if (r->slot && r->status != HAV_OK) r->slot->ready = false;
    if (r->slot) r->slot->busy = false;
    r->slot = nullptr;
    r->done = true;
    ++stats_.completed;
    stats_.points_done += r->n;
  }

  void worker_loop() {
    exec_.on_worker_start();
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      bool progress = false;
      // completed batches
      for (size_t f = 0; f < flights_.size(); ++f) {
        Flight& F = flights_[f];
        if (!F.busy) continue;
        const int q = exec_.query(static_cast<int>(f));
        if (q == 0) continue;
        for (RequestT* r : F.reqs) finish_request(r, q > 0 ? HAV_OK : HAV_ERR_HIP);
        F.reqs.clear();
        F.busy = false;
        progress = true;
      }
      // admission in arrival order; a request that does not fit yet keeps its place but
      // smaller ones behind it may pass
      for (auto it = pending_.begin(); it != pending_.end();) {
        SlotT* s = acquire_slot((*it)->n);
        if (!s) {
          ++it;
          continue;
        }
        (*it)->slot = s;
        admitted_.push_back(*it);
        it = pending_.erase(it);
        progress = true;
      }
      // launch everything admitted on a free flight
      if (!admitted_.empty()) {
        for (size_t f = 0; f < flights_.size(); ++f) {
          Flight& F = flights_[f];
          if (F.busy) continue;
          while (!admitted_.empty() && static_cast<int32_t>(F.reqs.size()) < max_batch_) {
            F.reqs.push_back(admitted_.front());
            admitted_.pop_front();
          }
          // The flight, its requests and their slots belong to this thread now (only the
          // worker looks at flights; submitters and pollers touch the queues and the
          // statistics), so the batch is enqueued without the lock.
          lk.unlock();
          const hav_status_t st = exec_.launch(static_cast<int>(f), F.reqs);
          if (st != HAV_OK) exec_.drain(static_cast<int>(f));
          lk.lock();
          ++stats_.batches;
          stats_.max_batch_seen = std::max<int64_t>(stats_.max_batch_seen, static_cast<int64_t>(F.reqs.size()));
          if (st != HAV_OK) {
            for (RequestT* r : F.reqs) finish_request(r, st);
            F.reqs.clear();
          } else {
            F.busy = true;
          }
          progress = true;
          break;
        }
      }
      bool inflight = false;
      for (const Flight& F : flights_) inflight |= F.busy;
      if (stop_ && !inflight && admitted_.empty()) break;
      if (!progress) {
        if (inflight)
          cv_.wait_for(lk, std::chrono::microseconds(10));
        else
          cv_.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
  }

  E exec_;
  size_t budget_ = 0, used_ = 0;
  int32_t max_batch_ = 0;
  std::vector<Flight> flights_;
  std::vector<std::unique_ptr<SlotT>> slots_;
  std::deque<RequestT*> pending_;   // submitted, no slot yet
  std::deque<RequestT*> admitted_;  // slot held, not launched yet
  std::unordered_map<uint64_t, std::unique_ptr<RequestT>> reqs_;
  uint64_t next_ticket_ = 1;
  hav_server_stats_t stats_{};
  std::mutex mu_;
  std::condition_variable cv_;
  std::thread worker_;
  bool stop_ = false;
  bool stopped_ = false;
};

}  // namespace hav_serve
