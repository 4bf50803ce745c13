// Host-only tests of the serving loop's scheduling core (server_core.hpp) with an executor
// over the CPU oracle, so no GPU is involved: result routing under continuous batching,
// queueing under a budget of one slot, release of idle slots of other classes, rejection
// of requests that can never fit, recovery of a slot after a failed batch, and shutdown
// with requests still queued. tests/test_serve_fake.py builds it with
// -fsanitize=address,undefined (and once with -fsanitize=thread), so the core and the
// oracle also run under the sanitizers. Exit status 0 when every case passes.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "../paper_2305_14306_amd/csrc/server_core.hpp"

// The oracle's C interface (oracle/hav_oracle.cpp), declared here as its Python wrapper does.
extern "C" {
typedef struct {
  int32_t layers;
  int32_t layer_ratio;
  int32_t t_max;
  int32_t flags;
  double sigma;
  float aspect[3];
  float fixed_voxel[3];
  int32_t select;
  uint32_t seed;
} OracleParams;
typedef struct {
  int32_t status;
  int32_t layers;
  float hi0;
  float mn[3];
  float mx[3];
  int32_t m[8];
  float s[8];
  int32_t evals[8];
  int32_t count[8];
  int32_t accepted[8];
  int32_t trimmed[8];
  int32_t padded[8];
} OracleInfo;
OracleParams oracle_params_default(void);
int32_t oracle_sample(const float* xyz, int64_t N, int64_t M, const OracleParams* p, int32_t* idx,
                      OracleInfo* info);
}

namespace {

int g_failures = 0;
#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__);    \
      std::printf(__VA_ARGS__);                           \
      std::printf("\n");                                  \
      ++g_failures;                                       \
    }                                                     \
  } while (0)

struct FakeMem {
  std::vector<int32_t> idx;
  hav_info_t info{};
};

// What the tests read back from the executor (the worker thread writes it).
struct FakeLog {
  std::atomic<int64_t> live_bytes{0}, max_live_bytes{0}, budget_violations{0};
  std::atomic<int64_t> inits{0}, launches{0}, allocs{0}, frees{0};
  std::atomic<int> busy_flights{0}, max_busy_flights{0};
  std::atomic<int> fail_launch_at{-1};  // launch number that fails at enqueue
  std::atomic<int> fail_query_at{-1};   // launch number whose completion reports failure
  int64_t budget = 0;
};

struct FakeExec {
  using SlotMem = FakeMem;
  using SlotT = hav_serve::Slot<FakeMem>;
  using RequestT = hav_serve::Request<FakeMem>;

  FakeLog* log = nullptr;
  int nflights = 2;
  size_t bytes_per_point = 64;
  size_t fixed = 1 << 20;
  int delay = 2;  // queries before a batch reports finished
  struct FlightState {
    int countdown = 0;
    bool fail = false;
  };
  std::vector<FlightState> fs;
  OracleParams op = oracle_params_default();

  size_t slot_bytes(int cls) const { return (size_t(1) << cls) * bytes_per_point; }
  size_t fixed_bytes() const { return fixed; }
  int flights() const { return nflights; }

  bool slot_alloc(SlotT& s) {
    s.mem.idx.assign(static_cast<size_t>(s.n_cap), -1);
    const int64_t live = log->live_bytes += static_cast<int64_t>(s.bytes);
    if (live + static_cast<int64_t>(fixed) > log->budget) ++log->budget_violations;
    int64_t m = log->max_live_bytes.load();
    while (live > m && !log->max_live_bytes.compare_exchange_weak(m, live)) {
    }
    ++log->allocs;
    return true;
  }

  void slot_free(SlotT& s) {
    log->live_bytes -= static_cast<int64_t>(s.bytes);
    s.mem.idx.clear();
    s.mem.idx.shrink_to_fit();
    ++log->frees;
  }

  hav_status_t launch(int f, const std::vector<RequestT*>& reqs) {
    if (fs.empty()) fs.resize(static_cast<size_t>(nflights));
    const int64_t k = log->launches++;
    if (k == log->fail_launch_at.load()) return HAV_ERR_HIP;
    for (RequestT* r : reqs) {
      SlotT* s = r->slot;
      if (!s->ready) {
        ++log->inits;
        s->ready = true;
      }
      if (r->n > s->n_cap) return HAV_ERR_WORKSPACE_TOO_SMALL;
      OracleInfo oi{};
      const int32_t st = oracle_sample(r->xyz_host, r->n, r->m, &op, s->mem.idx.data(), &oi);
      s->mem.info = hav_info_t{};
      s->mem.info.status = st;
    }
    fs[static_cast<size_t>(f)].countdown = delay;
    fs[static_cast<size_t>(f)].fail = (k == log->fail_query_at.load());
    const int b = ++log->busy_flights;
    int m = log->max_busy_flights.load();
    while (b > m && !log->max_busy_flights.compare_exchange_weak(m, b)) {
    }
    return HAV_OK;
  }

  int query(int f) {
    FlightState& F = fs[static_cast<size_t>(f)];
    if (F.countdown > 0) {
      --F.countdown;
      return 0;
    }
    --log->busy_flights;
    return F.fail ? -1 : 1;
  }

  void drain(int) {}

  void collect(RequestT& r) {
    r.info = r.slot->mem.info;
    r.status = static_cast<hav_status_t>(r.info.status);
    r.result.assign(r.slot->mem.idx.begin(), r.slot->mem.idx.begin() + r.m);
  }

  void on_worker_start() {}
};

using FakeServer = hav_serve::Server<FakeExec>;

// A seeded cloud (xorshift; uniform in a 20 m box, a quarter of the points in a 0.5 m blob).
std::vector<float> cloud(int64_t n, uint64_t seed) {
  std::vector<float> x(static_cast<size_t>(n) * 3);
  uint64_t s = seed * 0x9E3779B97F4A7C15ull + 1;
  auto u = [&]() {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return static_cast<float>((s >> 11) * (1.0 / 9007199254740992.0));
  };
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) x[static_cast<size_t>(3 * i + a)] = (i % 4 == 0) ? 0.5f * u() + 3.0f : 20.0f * u();
  return x;
}

std::vector<int32_t> alone(const std::vector<float>& x, int64_t n, int64_t m) {
  std::vector<int32_t> idx(static_cast<size_t>(m));
  OracleParams op = oracle_params_default();
  OracleInfo oi{};
  oracle_sample(x.data(), n, m, &op, idx.data(), &oi);
  return idx;
}

struct Job {
  std::vector<float> x;
  int64_t n, m;
  uint64_t ticket = 0;
  hav_status_t submit = HAV_OK;
};

// Submit every job, poll until each has finished; checks each result against the oracle
// alone. Returns the number of polled statuses that were not HAV_OK.
int run_jobs(FakeServer& S, std::vector<Job>& jobs, bool check_results) {
  for (Job& j : jobs) j.submit = S.submit(j.x.data(), j.n, j.m, &j.ticket);
  int not_ok = 0;
  for (Job& j : jobs) {
    if (j.submit != HAV_OK) continue;
    std::vector<int32_t> got(static_cast<size_t>(j.m));
    hav_info_t info{};
    double ms = 0.0;
    hav_status_t st;
    int spins = 0;
    while ((st = S.poll(j.ticket, got.data(), &info, &ms)) == HAV_NOT_READY) {
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      if (++spins > 200000) {
        CHECK(false, "request %llu never finished", static_cast<unsigned long long>(j.ticket));
        return not_ok + 1;
      }
    }
    if (st != HAV_OK) {
      ++not_ok;
      continue;
    }
    CHECK(ms >= 0.0, "latency %f", ms);
    if (check_results) CHECK(got == alone(j.x, j.n, j.m), "ticket %llu: result differs from the oracle alone",
                             static_cast<unsigned long long>(j.ticket));
    CHECK(S.poll(j.ticket, nullptr, nullptr, nullptr) == HAV_ERR_INVALID_ARG, "ticket not forgotten");
  }
  return not_ok;
}

FakeExec make_exec(FakeLog* log, int flights, int delay) {
  FakeExec e;
  e.log = log;
  e.nflights = flights;
  e.delay = delay;
  return e;
}

void case_routing() {
  // many mixed-size requests through continuous batching: every ticket gets its own result
  FakeLog log;
  log.budget = int64_t(1) << 40;
  FakeServer S(make_exec(&log, 2, 3), static_cast<size_t>(log.budget), 8);
  S.start();
  std::vector<Job> jobs;
  for (int i = 0; i < 40; ++i) {
    const int64_t n = 1000 + (i * 7919) % 19000;
    jobs.push_back(Job{cloud(n, 100 + i), n, std::max<int64_t>(1, n / (i % 2 ? 4 : 16))});
  }
  const int bad = run_jobs(S, jobs, true);
  CHECK(bad == 0, "routing: %d requests failed", bad);
  hav_server_stats_t st{};
  S.stats(&st);
  CHECK(st.completed == 40 && st.submitted == 40, "routing: completed %lld", static_cast<long long>(st.completed));
  CHECK(st.max_batch_seen > 1, "routing: no batch held more than one request");
  CHECK(st.batches < 40, "routing: %lld batches for 40 requests", static_cast<long long>(st.batches));
  CHECK(log.max_busy_flights.load() <= 2, "routing: %d flights busy at once", log.max_busy_flights.load());
  S.shutdown();
  CHECK(log.live_bytes.load() == 0 && log.allocs.load() == log.frees.load(), "routing: slots leaked");
}

void case_tiny_budget() {
  // a budget of one class-14 slot: requests queue and run one at a time, all correct
  FakeLog log;
  FakeExec e = make_exec(&log, 2, 1);
  log.budget = static_cast<int64_t>(e.fixed_bytes() + e.slot_bytes(14));
  FakeServer S(std::move(e), static_cast<size_t>(log.budget), 4);
  S.start();
  std::vector<Job> jobs;
  for (int i = 0; i < 12; ++i) {
    const int64_t n = 9000 + 500 * i;  // class 14 (8,193 .. 16,384 points)
    jobs.push_back(Job{cloud(n, 200 + i), n, n / 4});
  }
  const int bad = run_jobs(S, jobs, true);
  CHECK(bad == 0, "tiny budget: %d requests failed", bad);
  hav_server_stats_t st{};
  S.stats(&st);
  CHECK(st.slots_created == 1 && st.slots == 1, "tiny budget: %lld slots created",
        static_cast<long long>(st.slots_created));
  CHECK(st.max_batch_seen == 1, "tiny budget: batch of %lld", static_cast<long long>(st.max_batch_seen));
  CHECK(log.budget_violations.load() == 0, "tiny budget: budget exceeded");
  CHECK(log.inits.load() == 1, "tiny budget: slot initialised %lld times", static_cast<long long>(log.inits.load()));
  S.shutdown();
}

void case_eviction() {
  // room for one class-15 slot: requests alternate between classes 12 and 15, so idle
  // slots of the other class are released to make room; the budget is never exceeded
  FakeLog log;
  FakeExec e = make_exec(&log, 1, 1);
  log.budget = static_cast<int64_t>(e.fixed_bytes() + e.slot_bytes(15));
  FakeServer S(std::move(e), static_cast<size_t>(log.budget), 2);
  S.start();
  std::vector<Job> jobs;
  for (int i = 0; i < 8; ++i) {
    const int64_t n = (i % 2) ? 30000 : 3000;
    jobs.push_back(Job{cloud(n, 300 + i), n, n / 4});
  }
  const int bad = run_jobs(S, jobs, true);
  CHECK(bad == 0, "eviction: %d requests failed", bad);
  hav_server_stats_t st{};
  S.stats(&st);
  CHECK(st.evictions > 0, "eviction: no slot was released");
  CHECK(log.budget_violations.load() == 0, "eviction: budget exceeded");
  CHECK(static_cast<int64_t>(st.hbm_used) <= log.budget, "eviction: %llu bytes held",
        static_cast<unsigned long long>(st.hbm_used));
  S.shutdown();
  CHECK(log.live_bytes.load() == 0, "eviction: slots leaked");
}

void case_rejection() {
  // requests that can never fit, and invalid ones, are refused at submit; the rest run
  FakeLog log;
  FakeExec e = make_exec(&log, 1, 0);
  log.budget = static_cast<int64_t>(e.fixed_bytes() + e.slot_bytes(13));
  FakeServer S(std::move(e), static_cast<size_t>(log.budget), 4);
  S.start();
  std::vector<float> x = cloud(20000, 7);
  uint64_t t = 0;
  CHECK(S.submit(x.data(), 20000, 5000, &t) == HAV_ERR_OUT_OF_MEMORY, "class 15 in a class-13 budget accepted");
  CHECK(S.submit(x.data(), int64_t(1) << 25, 10, &t) == HAV_ERR_INVALID_ARG, "N above the largest class accepted");
  CHECK(S.submit(x.data(), 100, 101, &t) == HAV_ERR_INVALID_ARG, "M > N accepted");
  CHECK(S.submit(x.data(), 100, 0, &t) == HAV_ERR_INVALID_ARG, "M = 0 accepted");
  CHECK(S.submit(nullptr, 100, 10, &t) == HAV_ERR_INVALID_ARG, "null cloud accepted");
  CHECK(S.submit(x.data(), 100, 10, nullptr) == HAV_ERR_INVALID_ARG, "null ticket accepted");
  CHECK(S.poll(12345, nullptr, nullptr, nullptr) == HAV_ERR_INVALID_ARG, "unknown ticket answered");
  std::vector<Job> jobs;
  jobs.push_back(Job{cloud(8000, 8), 8000, 2000});
  jobs.push_back(Job{cloud(50, 9), 50, 50});  // M == N
  const int bad = run_jobs(S, jobs, true);
  CHECK(bad == 0, "rejection: %d valid requests failed", bad);
  S.shutdown();
}

void case_failure_recovery() {
  // the second batch fails at enqueue and the fourth reports failure on completion: their
  // requests get HAV_ERR_HIP, their slots are initialised again before the next request,
  // and every other request is exact
  FakeLog log;
  FakeExec e = make_exec(&log, 1, 1);
  log.budget = static_cast<int64_t>(e.fixed_bytes() + e.slot_bytes(13));
  log.fail_launch_at = 1;
  log.fail_query_at = 3;
  FakeServer S(std::move(e), static_cast<size_t>(log.budget), 1);
  S.start();
  std::vector<Job> jobs;
  for (int i = 0; i < 6; ++i) jobs.push_back(Job{cloud(5000, 400 + i), 5000, 1250});
  // submit and poll one at a time so that batch k is request k
  int failed = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    std::vector<Job> one(1, jobs[i]);
    failed += run_jobs(S, one, true);
  }
  CHECK(failed == 2, "failure: %d requests failed, expected 2", failed);
  CHECK(log.inits.load() == 3, "failure: slot initialised %lld times, expected 3",
        static_cast<long long>(log.inits.load()));
  S.shutdown();
}

void case_shutdown_with_queue() {
  // shutting down with requests queued behind a one-slot budget drops them cleanly
  FakeLog log;
  FakeExec e = make_exec(&log, 1, 50);
  log.budget = static_cast<int64_t>(e.fixed_bytes() + e.slot_bytes(12));
  std::vector<std::vector<float>> xs;
  for (int i = 0; i < 16; ++i) xs.push_back(cloud(3000, 500 + i));
  {
    FakeServer S(std::move(e), static_cast<size_t>(log.budget), 1);
    S.start();
    uint64_t t = 0;
    for (auto& x : xs) CHECK(S.submit(x.data(), 3000, 100, &t) == HAV_OK, "submit refused");
    S.shutdown();
  }
  CHECK(log.live_bytes.load() == 0 && log.allocs.load() == log.frees.load(), "shutdown: slots leaked");
}

}  // namespace

int main() {
  const std::pair<const char*, void (*)()> cases[] = {
      {"routing", case_routing},           {"tiny budget", case_tiny_budget},
      {"eviction", case_eviction},         {"rejection", case_rejection},
      {"failure recovery", case_failure_recovery}, {"shutdown with queue", case_shutdown_with_queue}};
  for (const auto& c : cases) {
    std::printf("case %s\n", c.first);
    std::fflush(stdout);
    const int before = g_failures;
    c.second();
    std::printf("case %s: %s\n", c.first, g_failures == before ? "pass" : "FAIL");
    std::fflush(stdout);
  }
  if (g_failures == 0) std::printf("ALL PASS\n");
  return g_failures == 0 ? 0 : 1;
}
