// Scheduling core of the serving runtime (stap_server_*): an HBM arena,
// admission of frames in arrival order while their buffers fit, fair-share
// slicing of the active frames into steps, and a pipeline of up to two steps
// in flight on one compute queue.
//
// The core holds no device code and makes no HIP call: every device action
// goes through the Exec interface, so the same scheduler runs against the HIP
// executor of the library and against a CPU fake in the tests (admission,
// slicing, failure handling, memory reuse).
//
// Invariants:
//   * a frame's arena range is released only when no slice of it is in
//     flight (after the steps holding its slices have completed, or after the
//     executor has drained the compute queue following a failure);
//   * a frame record is deleted only by wait(), after it reached kDone or
//     kFailed, and no in-flight step refers to it any more;
//   * step slots are reused only after their step has completed, so the
//     executor may keep per-slot tables in host staging memory.
#ifndef KSTAP_SCHED_H_
#define KSTAP_SCHED_H_

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/kstap.h"

namespace kstap {
namespace sched {

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device arena (offsets, 256-byte granules).
class Arena {
 public:
  explicit Arena(size_t bytes) : size_(bytes) { free_[0] = bytes; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (const auto& kv : free_) s += kv.second;
    return s;
  }
  size_t size() const { return size_; }
  static size_t round(size_t b) { return (b + 255) / 256 * 256; }

 private:
  size_t size_;
  std::map<size_t, size_t> free_;
};

enum FrameState { kPending = 0, kUploading, kComputing, kDownloading, kDone, kFailed };

struct Frame {
  uint64_t ticket = 0;
  size_t bytes = 0;       // device bytes (arena)
  size_t off = 0;         // arena offset once admitted
  int64_t npos = 0;       // work positions (a multiple of the chain length)
  int64_t pixels = 0;     // pixels credited when the frame completes
  int64_t cursor = 0;     // positions handed to steps
  int64_t done = 0;       // positions whose step has completed
  int inflight = 0;       // slices in steps that have not completed
  int state = kPending;
  stap_status status = STAP_OK;
  double t_submit = 0, t_done = 0;
  void* exec = nullptr;   // executor data of the frame
};

struct Slice {
  Frame* f;
  int64_t first, end;     // positions [first, end)
};

// Device side.  Every call is made from the worker thread.
class Exec {
 public:
  enum Poll { kReady = 0, kNotReady = 1, kError = 2 };
  virtual ~Exec() = default;
  // enqueue the frame's input (copy, split) into its arena range; false on error
  virtual bool upload(Frame* f) = 0;
  virtual Poll upload_state(Frame* f) = 0;
  // enqueue one step (slot 0 or 1); false on error (nothing may be running from it
  // afterwards except what drain() waits for)
  virtual bool launch(int slot, const std::vector<Slice>& slices) = 0;
  virtual Poll step_state(int slot) = 0;
  // enqueue the copy of the frame's results out of its arena range
  virtual bool download(Frame* f) = 0;
  virtual Poll download_state(Frame* f) = 0;
  // blocks until all enqueued compute work has finished (or failed)
  virtual void drain() = 0;
  // frees the executor data of a frame record
  virtual void forget(Frame* f) = 0;
  virtual std::string error() = 0;
  // called once on the worker thread before any other call (binds the device)
  virtual bool thread_init() { return true; }
};

// Fair-share slices of one step over the ready frames (arrival order): each
// frame gets up to `min_slice` positions, then the rest of the step budget
// goes to the oldest frames first, so a small frame finishes in one step and
// a large one is not stretched by the number of frames beside it.  Slices
// are multiples of `chain` positions (or end the frame).
inline void plan_slices(const std::vector<Frame*>& ready, int64_t step_positions, int64_t chain,
                        std::vector<Slice>* out) {
  out->clear();
  auto up = [chain](int64_t v) { return (v + chain - 1) / chain * chain; };
  const int64_t min_slice = up(std::max<int64_t>(16384, step_positions / 16));
  int64_t budget = step_positions;
  std::vector<int64_t> take(ready.size());
  for (size_t i = 0; i < ready.size(); ++i) {
    take[i] = std::min(ready[i]->npos - ready[i]->cursor, min_slice);
    budget -= take[i];
  }
  for (size_t i = 0; i < ready.size() && budget > 0; ++i) {
    const int64_t extra = std::min(ready[i]->npos - ready[i]->cursor - take[i], up(budget));
    take[i] += extra;
    budget -= extra;
  }
  for (size_t i = 0; i < ready.size(); ++i)
    if (take[i] > 0) out->push_back({ready[i], ready[i]->cursor, ready[i]->cursor + take[i]});
}

struct Config {
  size_t budget = 0;
  int max_inflight = 16;
  int64_t step_positions = int64_t(1) << 20;
  int64_t chain = 16;
  int max_slices = 16;    // slices per step (the executor's table capacity)
};

class Scheduler {
 public:
  static constexpr int kSlots = 2;

  Scheduler(const Config& cfg, Exec* exec) : cfg_(cfg), exec_(exec), arena_(cfg.budget) {}
  ~Scheduler() { stop(); }

  void start() { worker_ = std::thread([this]() { loop(); }); }

  // Finishes every queued frame, then joins the worker.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    if (worker_.joinable()) worker_.join();
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : frames_) {
      exec_->forget(kv.second);
      delete kv.second;
    }
    frames_.clear();
  }

  // Takes ownership of f (bytes, npos, pixels and exec filled in).
  stap_status submit(Frame* f, uint64_t* ticket, std::string* err) {
    if (f->bytes > cfg_.budget) {
      *err = "frame needs " + std::to_string(f->bytes) + " bytes of device memory, the budget is " +
             std::to_string(cfg_.budget);
      return STAP_ERR_BUSY;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) {
        *err = "server is shutting down";
        return STAP_ERR_INVALID_ARG;
      }
      f->ticket = next_ticket_++;
      f->t_submit = now_s();
      if (t_first_ < 0) t_first_ = f->t_submit;
      frames_[f->ticket] = f;
      pending_.push_back(f);
      *ticket = f->ticket;
    }
    cv_work_.notify_all();
    return STAP_OK;
  }

  stap_status wait(uint64_t ticket, int timeout_ms, double* latency_s, std::string* err) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = frames_.find(ticket);
    if (it == frames_.end()) {
      *err = "unknown ticket " + std::to_string(ticket);
      return STAP_ERR_INVALID_ARG;
    }
    Frame* f = it->second;
    auto done = [f]() { return f->state == kDone || f->state == kFailed; };
    if (timeout_ms < 0) {
      cv_done_.wait(lk, done);
    } else if (!cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
      *err = "frame " + std::to_string(ticket) + " not finished within " + std::to_string(timeout_ms) + " ms";
      return STAP_ERR_BUSY;
    }
    const stap_status st = f->status;
    if (latency_s) *latency_s = f->t_done - f->t_submit;
    frames_.erase(it);
    exec_->forget(f);
    delete f;
    if (st != STAP_OK) *err = "frame " + std::to_string(ticket) + " failed: " + fatal_;
    return st;
  }

  void stats(double* p50, double* p99, double* pixels_per_s, int64_t* frames_done) {
    std::lock_guard<std::mutex> lk(mu_);
    std::vector<double> l = latencies_;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) -> double {
      if (l.empty()) return 0.0;
      const size_t i = std::min(l.size() - 1, size_t(q * double(l.size() - 1) + 0.5));
      return l[i];
    };
    if (p50) *p50 = pct(0.50);
    if (p99) *p99 = pct(0.99);
    if (pixels_per_s) *pixels_per_s = (t_last_ > t_first_) ? double(pixels_done_) / (t_last_ - t_first_) : 0.0;
    if (frames_done) *frames_done = int64_t(l.size());
  }

  // test hooks
  size_t arena_free() {
    std::lock_guard<std::mutex> lk(mu_);
    return arena_.free_bytes();
  }
  int64_t steps_launched() {
    std::lock_guard<std::mutex> lk(mu_);
    return steps_launched_;
  }

 private:
  struct Step {
    bool busy = false;
    int64_t seq = 0;
    std::vector<Slice> slices;
  };

  void finish_locked(Frame* f, stap_status st, const std::string& what) {
    if (f->state == kDone || f->state == kFailed) return;
    f->status = st;
    f->state = (st == STAP_OK) ? kDone : kFailed;
    f->t_done = now_s();
    if (st == STAP_OK) {
      latencies_.push_back(f->t_done - f->t_submit);
      pixels_done_ += f->pixels;
      t_last_ = f->t_done;
    } else {
      fatal_ = what;
    }
    arena_.release(f->off, f->bytes);
    active_.erase(std::remove(active_.begin(), active_.end(), f), active_.end());
    cv_done_.notify_all();
  }

  void admit_locked() {
    while (dead_ && !pending_.empty()) {   // the worker cannot use the device: every frame fails
      Frame* f = pending_.front();
      pending_.pop_front();
      f->status = STAP_ERR_DEVICE;
      f->state = kFailed;
      f->t_done = now_s();
      cv_done_.notify_all();
    }
    while (!pending_.empty() && int(active_.size()) < cfg_.max_inflight) {
      Frame* f = pending_.front();
      size_t off = 0;
      if (!arena_.alloc(f->bytes, &off)) break;
      pending_.pop_front();
      f->off = off;
      active_.push_back(f);
      f->state = kUploading;
      if (!exec_->upload(f)) finish_locked(f, STAP_ERR_DEVICE, exec_->error());   // nothing of it runs
    }
  }

  void poll_locked() {
    const std::vector<Frame*> act = active_;   // finish_locked edits active_
    for (Frame* f : act) {
      if (f->state == kUploading) {
        const Exec::Poll p = exec_->upload_state(f);
        if (p == Exec::kReady) f->state = kComputing;
        else if (p == Exec::kError) finish_locked(f, STAP_ERR_DEVICE, exec_->error());
      } else if (f->state == kDownloading) {
        const Exec::Poll p = exec_->download_state(f);
        if (p == Exec::kReady) finish_locked(f, STAP_OK, std::string());
        else if (p == Exec::kError) finish_locked(f, STAP_ERR_DEVICE, exec_->error());
      }
    }
  }

  // A completed step: its slices are done; frames whose last slice it held
  // start their download.
  void retire_locked(Step& s) {
    for (const Slice& sl : s.slices) {
      Frame* f = sl.f;
      --f->inflight;
      if (f->state != kComputing) continue;   // failed meanwhile
      f->done = std::max(f->done, sl.end);
      if (f->done >= f->npos && f->inflight == 0) {
        if (exec_->download(f)) f->state = kDownloading;
        else finish_locked(f, STAP_ERR_DEVICE, exec_->error());
      }
    }
    s.slices.clear();
    s.busy = false;
  }

  // After a failed launch or a failed step: wait for whatever is still
  // running, then fail the frames of the steps that did not complete.
  void recover_locked(std::unique_lock<std::mutex>& lk, int bad_slot) {
    lk.unlock();
    exec_->drain();
    lk.lock();
    const std::string what = exec_->error();
    for (int k = 0; k < kSlots; ++k) {
      Step& s = steps_[k];
      if (!s.busy) continue;
      const bool ok = k != bad_slot && exec_->step_state(k) == Exec::kReady;
      if (ok) {
        retire_locked(s);
        continue;
      }
      for (const Slice& sl : s.slices) --sl.f->inflight;
      for (const Slice& sl : s.slices) finish_locked(sl.f, STAP_ERR_DEVICE, what);
      s.slices.clear();
      s.busy = false;
    }
  }

  void loop() {
    const bool bound = exec_->thread_init();
    std::unique_lock<std::mutex> lk(mu_);
    if (!bound) {
      dead_ = true;
      fatal_ = exec_->error();
    }
    std::vector<Slice> slices;
    while (true) {
      admit_locked();
      poll_locked();
      // retire completed steps, oldest first (one compute queue: in order)
      bool progressed = false;
      while (true) {
        int oldest = -1;
        for (int k = 0; k < kSlots; ++k)
          if (steps_[k].busy && (oldest < 0 || steps_[k].seq < steps_[oldest].seq)) oldest = k;
        if (oldest < 0) break;
        const Exec::Poll p = exec_->step_state(oldest);
        if (p == Exec::kNotReady) break;
        if (p == Exec::kError) {
          recover_locked(lk, oldest);
        } else {
          retire_locked(steps_[oldest]);
        }
        progressed = true;
      }
      // enqueue the next step while the previous one runs
      int free_slot = -1;
      for (int k = 0; k < kSlots; ++k)
        if (!steps_[k].busy) free_slot = k;
      std::vector<Frame*> ready;
      for (Frame* f : active_)
        if (f->state == kComputing && f->cursor < f->npos && int(ready.size()) < cfg_.max_slices)
          ready.push_back(f);
      if (free_slot >= 0 && !ready.empty()) {
        plan_slices(ready, cfg_.step_positions, cfg_.chain, &slices);
        Step& s = steps_[free_slot];
        s.busy = true;
        s.seq = ++seq_;
        s.slices = slices;
        for (const Slice& sl : slices) {
          sl.f->cursor = sl.end;
          ++sl.f->inflight;
        }
        ++steps_launched_;
        lk.unlock();
        const bool ok = exec_->launch(free_slot, slices);
        lk.lock();
        if (!ok) recover_locked(lk, free_slot);
        continue;
      }
      if (progressed) continue;
      const bool steps_busy = steps_[0].busy || steps_[1].busy;
      if (stop_ && pending_.empty() && active_.empty() && !steps_busy) break;
      cv_work_.wait_for(lk, std::chrono::microseconds(steps_busy ? 50 : 200));
    }
  }

  Config cfg_;
  Exec* exec_;
  Arena arena_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Frame*> pending_;
  std::vector<Frame*> active_;
  std::map<uint64_t, Frame*> frames_;
  Step steps_[kSlots];
  int64_t seq_ = 0, steps_launched_ = 0;
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  bool dead_ = false;
  std::thread worker_;
  std::vector<double> latencies_;
  int64_t pixels_done_ = 0;
  double t_first_ = -1, t_last_ = -1;
  std::string fatal_;
};

}  // namespace sched
}  // namespace kstap

#endif  // KSTAP_SCHED_H_
