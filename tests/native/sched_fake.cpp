// CPU test driver of the serving scheduler (paper_1604_03622_amd/csrc/kstap_sched.h)
// against a fake executor: two worker threads play the copy and the compute
// queues, an ownership map of the arena's 256-byte granules catches memory
// reused while work on it is still queued or running, and every work
// position of every frame is counted.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_server_sched_cpu.py.
//
// Each scenario prints "ok <name>"; any violated check prints "FAIL ..." and
// exits with status 1.
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_1604_03622_amd/csrc/kstap_sched.h"

namespace ks = kstap::sched;

#define CHECK(c, ...)                                        \
  do {                                                       \
    if (!(c)) {                                              \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                     \
      std::fprintf(stderr, "\n");                            \
      std::exit(1);                                          \
    }                                                        \
  } while (0)

// one in-order queue of work run by its own thread
class Queue {
 public:
  Queue() : th_([this]() { run(); }) {}
  ~Queue() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    th_.join();
  }
  void push(std::function<void()> fn) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      q_.push_back(std::move(fn));
      ++pushed_;
    }
    cv_.notify_all();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [this]() { return done_ == pushed_; });
  }

 private:
  void run() {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      cv_.wait(lk, [this]() { return stop_ || !q_.empty(); });
      if (q_.empty() && stop_) return;
      auto fn = std::move(q_.front());
      q_.pop_front();
      lk.unlock();
      fn();
      lk.lock();
      ++done_;
      cv_.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> q_;
  uint64_t pushed_ = 0, done_ = 0;
  bool stop_ = false;
  std::thread th_;
};

struct FakeFrame {
  uint64_t id = 0;                   // submission index (the ticket is assigned later)
  std::vector<int> count;            // times each position was computed
  std::atomic<int> pending{0};       // enqueued device operations not yet run
  std::atomic<bool> up{false}, down{false}, up_fail{false};
  bool downloaded = false;
};

class FakeExec : public ks::Exec {
 public:
  explicit FakeExec(size_t budget, unsigned seed) : owner_(budget / 256, nullptr), rng_(seed) {}
  ~FakeExec() override {
    copy_.drain();
    comp_.drain();
  }

  int64_t fail_launch_at = -1;       // step index whose launch is refused
  int64_t fail_step_at = -1;         // step index that reports a device error after running
  uint64_t fail_upload_id = ~0ull;   // frame whose upload is refused
  std::atomic<int64_t> steps{0};
  std::atomic<int> max_frames_in_step{0};

  bool upload(ks::Frame* f) override {
    FakeFrame* ff = ff_of(f);
    if (ff->id == fail_upload_id) {
      err_ = "injected upload failure";
      return false;
    }
    ++ff->pending;
    const size_t off = f->off, bytes = ks::Arena::round(f->bytes);
    const int us = int(rng() % 200);
    copy_.push([this, ff, off, bytes, us]() {
      std::this_thread::sleep_for(std::chrono::microseconds(us));
      std::lock_guard<std::mutex> lk(own_mu_);
      for (size_t g = off / 256; g < (off + bytes) / 256; ++g) {
        FakeFrame* prev = owner_[g];
        CHECK(prev == nullptr || prev == ff || prev->pending.load() == 0,
              "arena granule %zu overwritten while frame %llu still has %d queued operations", g,
              (unsigned long long)prev->id, prev->pending.load());
        owner_[g] = ff;
      }
      ff->up = true;
      --ff->pending;
    });
    return true;
  }
  Poll upload_state(ks::Frame* f) override { return ff_of(f)->up ? kReady : kNotReady; }

  bool launch(int slot, const std::vector<ks::Slice>& slices) override {
    const int64_t idx = steps++;
    if (idx == fail_launch_at) {
      err_ = "injected launch failure";
      return false;
    }
    int cur = max_frames_in_step.load();
    while (int(slices.size()) > cur && !max_frames_in_step.compare_exchange_weak(cur, int(slices.size()))) {
    }
    step_done_[slot] = false;
    step_err_[slot] = false;
    const bool fault = idx == fail_step_at;
    struct Work {
      FakeFrame* ff;
      size_t off, bytes;
      int64_t first, end;
    };
    std::vector<Work> work;
    for (const ks::Slice& s : slices) {
      FakeFrame* ff = ff_of(s.f);
      CHECK(s.first >= 0 && s.end <= s.f->npos && s.first < s.end, "bad slice [%lld, %lld) of %lld",
            (long long)s.first, (long long)s.end, (long long)s.f->npos);
      CHECK(s.first % 16 == 0 && (s.end % 16 == 0 || s.end == s.f->npos), "slice off the chain grid");
      ++ff->pending;
      work.push_back({ff, s.f->off, ks::Arena::round(s.f->bytes), s.first, s.end});
    }
    const int us = int(rng() % 300);
    comp_.push([this, work, slot, fault, us]() {
      std::this_thread::sleep_for(std::chrono::microseconds(us));
      for (const Work& w : work) {
        {
          std::lock_guard<std::mutex> lk(own_mu_);
          for (size_t g = w.off / 256; g < (w.off + w.bytes) / 256; ++g)
            CHECK(owner_[g] == w.ff, "slice of frame %llu runs on memory owned by another frame",
                  (unsigned long long)w.ff->id);
        }
        for (int64_t p = w.first; p < w.end; ++p) ++w.ff->count[p];
        --w.ff->pending;
      }
      if (fault) step_err_[slot] = true;
      step_done_[slot] = true;
    });
    return true;
  }
  Poll step_state(int slot) override {
    if (!step_done_[slot]) return kNotReady;
    if (step_err_[slot]) {
      err_ = "injected device error";
      return kError;
    }
    return kReady;
  }

  bool download(ks::Frame* f) override {
    FakeFrame* ff = ff_of(f);
    ++ff->pending;
    copy_.push([ff]() {
      ff->downloaded = true;
      ff->down = true;
      --ff->pending;
    });
    return true;
  }
  Poll download_state(ks::Frame* f) override { return ff_of(f)->down ? kReady : kNotReady; }

  void drain() override { comp_.drain(); }
  void forget(ks::Frame* f) override { f->exec = nullptr; }
  std::string error() override { return err_; }

  static FakeFrame* ff_of(ks::Frame* f) { return static_cast<FakeFrame*>(f->exec); }
  unsigned rng() {
    std::lock_guard<std::mutex> lk(rng_mu_);
    return unsigned(rng_());
  }

 private:
  std::mutex own_mu_, rng_mu_;
  std::vector<FakeFrame*> owner_;
  std::mt19937 rng_;
  std::atomic<bool> step_done_[ks::Scheduler::kSlots] = {{true}, {true}};
  std::atomic<bool> step_err_[ks::Scheduler::kSlots] = {{false}, {false}};
  std::string err_;
  Queue copy_, comp_;
};

struct Run {
  std::vector<FakeFrame*> frames;
  std::vector<uint64_t> tickets;
  std::vector<stap_status> status;
};

// Submits `n` frames (sizes drawn from rng) with small random gaps and waits
// for each; returns per-frame statuses.
Run submit_all(ks::Scheduler& s, FakeExec& ex, int n, size_t max_bytes, std::mt19937& rng, int gap_us = 100,
               uint64_t id_base = 0) {
  Run r;
  for (int i = 0; i < n; ++i) {
    FakeFrame* ff = new FakeFrame();
    ff->id = id_base + uint64_t(i);
    const int64_t npos = 16 * int64_t(1 + rng() % 4096);
    ff->count.assign(size_t(npos), 0);
    ks::Frame* f = new ks::Frame();
    f->npos = npos;
    f->pixels = npos;
    f->bytes = 256 + rng() % max_bytes;
    f->exec = ff;
    uint64_t t = 0;
    std::string err;
    const stap_status st = s.submit(f, &t, &err);
    CHECK(st == STAP_OK, "submit failed: %s", err.c_str());
    r.frames.push_back(ff);
    r.tickets.push_back(t);
    if (gap_us) std::this_thread::sleep_for(std::chrono::microseconds(rng() % gap_us));
  }
  for (size_t i = 0; i < r.tickets.size(); ++i) {
    double lat = 0;
    std::string err;
    r.status.push_back(s.wait(r.tickets[i], -1, &lat, &err));
  }
  (void)ex;
  return r;
}

void check_complete(const Run& r, const char* what, bool all_ok) {
  for (size_t i = 0; i < r.frames.size(); ++i) {
    FakeFrame* ff = r.frames[i];
    if (r.status[i] != STAP_OK) {
      CHECK(!all_ok, "%s: frame %zu failed", what, i);
      continue;
    }
    CHECK(ff->downloaded, "%s: frame %zu completed without its download", what, i);
    for (size_t p = 0; p < ff->count.size(); ++p)
      CHECK(ff->count[p] == 1, "%s: frame %zu position %zu computed %d times", what, i, p, ff->count[p]);
  }
}

void free_run(Run& r) {
  for (FakeFrame* ff : r.frames) {
    CHECK(ff->pending.load() == 0, "frame %llu left queued operations", (unsigned long long)ff->id);
    delete ff;
  }
  r.frames.clear();
}

ks::Config config(size_t budget, int inflight, int64_t step) {
  ks::Config c;
  c.budget = budget;
  c.max_inflight = inflight;
  c.max_slices = inflight;
  c.step_positions = step;
  c.chain = 16;
  return c;
}

void scenario_mixed_stream() {
  const size_t budget = size_t(64) << 20;
  FakeExec ex(budget, 1);
  ks::Scheduler s(config(budget, 8, 8192), &ex);
  s.start();
  std::mt19937 rng(11);
  Run r = submit_all(s, ex, 300, budget / 3, rng);
  check_complete(r, "mixed stream", true);
  double p50, p99, pps;
  int64_t nf;
  s.stats(&p50, &p99, &pps, &nf);
  CHECK(nf == 300 && p99 >= p50 && p50 > 0 && pps > 0, "stats: %lld frames p50 %g p99 %g", (long long)nf, p50, p99);
  CHECK(ex.max_frames_in_step.load() <= 8 && ex.max_frames_in_step.load() > 1, "frames per step %d",
        ex.max_frames_in_step.load());
  s.stop();
  CHECK(s.arena_free() == budget, "arena not free after the run");
  free_run(r);
  std::printf("ok mixed_stream steps=%lld\n", (long long)ex.steps.load());
}

void scenario_busy_refusal() {
  const size_t budget = size_t(1) << 20;
  FakeExec ex(budget, 2);
  ks::Scheduler s(config(budget, 4, 4096), &ex);
  s.start();
  ks::Frame* f = new ks::Frame();
  FakeFrame ff;
  f->npos = 16;
  f->bytes = budget + 1;
  f->exec = &ff;
  uint64_t t = 0;
  std::string err;
  CHECK(s.submit(f, &t, &err) == STAP_ERR_BUSY, "an oversized frame was admitted");
  delete f;
  // a frame of exactly the budget fits (alone)
  std::mt19937 rng(3);
  Run r = submit_all(s, ex, 5, budget, rng);
  check_complete(r, "busy", true);
  s.stop();
  free_run(r);
  std::printf("ok busy_refusal\n");
}

void scenario_failure(const char* name, int64_t launch_at, int64_t step_at, uint64_t upload_id) {
  const size_t budget = size_t(32) << 20;
  FakeExec ex(budget, 5);
  ex.fail_launch_at = launch_at;
  ex.fail_step_at = step_at;
  ex.fail_upload_id = upload_id;
  ks::Scheduler s(config(budget, 6, 4096), &ex);
  s.start();
  std::mt19937 rng(7);
  Run r = submit_all(s, ex, 60, budget / 4, rng);
  int failed = 0;
  for (auto st : r.status) failed += st != STAP_OK;
  CHECK(failed >= 1, "%s: no frame failed", name);
  CHECK(failed < 60, "%s: every frame failed", name);
  check_complete(r, name, false);
  // the server keeps serving after the failure
  Run r2 = submit_all(s, ex, 20, budget / 4, rng, 100, 1000);
  check_complete(r2, name, true);
  s.stop();
  CHECK(s.arena_free() == budget, "%s: arena not free after the run", name);
  free_run(r);
  free_run(r2);
  std::printf("ok %s failed=%d\n", name, failed);
}

void scenario_destroy_with_open_tickets() {
  const size_t budget = size_t(16) << 20;
  FakeExec ex(budget, 9);
  std::vector<FakeFrame*> keep;
  {
    ks::Scheduler s(config(budget, 4, 4096), &ex);
    s.start();
    std::mt19937 rng(9);
    for (int i = 0; i < 20; ++i) {
      FakeFrame* ff = new FakeFrame();
      ff->id = uint64_t(i);
      ff->count.assign(16 * (1 + rng() % 256), 0);
      ks::Frame* f = new ks::Frame();
      f->npos = int64_t(ff->count.size());
      f->bytes = 256 + rng() % (budget / 4);
      f->exec = ff;
      uint64_t t;
      std::string err;
      CHECK(s.submit(f, &t, &err) == STAP_OK, "submit");
      keep.push_back(ff);
    }
    s.stop();   // finishes every frame, releases the tickets
    CHECK(s.arena_free() == budget, "arena not free after stop");
  }
  for (FakeFrame* ff : keep) {
    CHECK(ff->downloaded, "frame %llu not finished by stop", (unsigned long long)ff->id);
    for (int c : ff->count) CHECK(c == 1, "position computed %d times", c);
    delete ff;
  }
  std::printf("ok destroy_with_open_tickets\n");
}

void scenario_slicing_policy() {
  std::vector<ks::Frame> fr(5);
  const int64_t sizes[5] = {4096 * 16, 64, 160000, 16, 1 << 20};
  std::vector<ks::Frame*> ready;
  for (int i = 0; i < 5; ++i) {
    fr[i].npos = sizes[i];
    fr[i].cursor = 0;
    ready.push_back(&fr[i]);
  }
  std::vector<ks::Slice> out;
  ks::plan_slices(ready, 1 << 20, 16, &out);
  CHECK(out.size() == 5, "every ready frame gets a slice");
  int64_t tot = 0;
  for (const auto& s : out) {
    CHECK(s.first == 0 && (s.end % 16 == 0 || s.end == s.f->npos), "alignment");
    CHECK(s.end <= s.f->npos, "slice past the frame");
    tot += s.end - s.first;
  }
  CHECK(tot <= (1 << 20) + 16, "step budget exceeded: %lld", (long long)tot);
  CHECK(out[1].end == 64 && out[3].end == 16, "small frames finish in one step");
  CHECK(out[0].end == 4096 * 16 && out[2].end == 160000, "older frames take the rest of the budget first");
  CHECK(out[4].end >= 65536, "every frame gets at least the minimum slice");
  std::printf("ok slicing_policy\n");
}

int main() {
  scenario_slicing_policy();
  scenario_mixed_stream();
  scenario_busy_refusal();
  scenario_failure("launch_failure", 5, -1, ~0ull);
  scenario_failure("device_error", -1, 7, ~0ull);
  scenario_failure("upload_failure", -1, -1, 3);
  scenario_destroy_with_open_tickets();
  std::printf("all scenarios passed\n");
  return 0;
}
