// Serving: frames of mixed sizes admitted by HBM budget and processed with
// continuous batching.  See the stap_server_* declarations in kstap.h.
//
// One worker thread owns the device work.  Each scheduling step takes a
// fair-share slice of every active frame (a row-major pixel range), numbers
// the slices' work items longest first per kernel class and runs them in one
// persistent launch per class on the compute stream.  While a step runs, the
// worker admits waiting frames in arrival order as soon as their buffers fit
// in the HBM arena (their host-to-device copies go on a separate copy stream
// and overlap the step) and finishes frames whose last slice is done (results
// copied back on the copy stream).  New frames join at the next step, so a
// small frame never waits behind a large one for longer than one step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "kstap_host.h"
#include "kstap_internal.h"

using namespace kstap::host;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device arena (offsets, 256-byte granules).
class Arena {
 public:
  explicit Arena(size_t bytes) { free_[0] = bytes; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
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
    bytes = (bytes + 255) / 256 * 256;
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

 private:
  std::map<size_t, size_t> free_;
};

enum FrameState { kPending = 0, kUploading, kComputing, kDownloading, kDone, kFailed };

struct Frame {
  uint64_t ticket = 0;
  const stap_plan_s* plan = nullptr;
  const void* x_src = nullptr;
  bool x_on_device = false;
  int H = 0, W = 0;
  float* T_out = nullptr;
  uint8_t* D_out = nullptr;
  int cls = -1;
  size_t off = 0, bytes = 0, x_bytes = 0;
  bool planes = false;     // mixed path: split planes at off + planes_off
  size_t planes_off = 0;
  int64_t cursor = 0, total = 0, inflight_end = 0;   // cursor/inflight_end/npos: tiled-order positions
  int64_t npos = 0;
  double t_submit = 0, t_done = 0;
  int state = kPending;
  stap_status status = STAP_OK;
  hipEvent_t ev_up = nullptr, ev_down = nullptr;
};

// Device bytes of one frame: [x, unless it is already on the device] [T] [D]
// [split planes of the mixed path, if its kernel reads them].
size_t frame_bytes(const stap_plan_s* pl, int H, int W, bool x_on_device, size_t* x_bytes, size_t* planes_off) {
  const stap_config& c = pl->cfg;
  const size_t px = size_t(H) * W;
  *x_bytes = x_on_device ? 0 : px * c.p * c.q * 8;
  *planes_off = (*x_bytes + 255) / 256 * 256 + (px * 4 + 255) / 256 * 256 + (px + 255) / 256 * 256;
  const size_t planes = kstap::kernel_needs_planes(c.p, c.q, c.r_b, c.precision) ? px * c.p * c.q * 8 : 0;
  return *planes_off + (planes + 255) / 256 * 256;
}

}  // namespace

struct stap_server_s {
  size_t budget = 0;
  int max_inflight = 0;
  int64_t step_pixels = 0;
  int device = 0;
  char* arena_base = nullptr;
  Arena* arena = nullptr;
  hipStream_t s_copy = nullptr, s_comp = nullptr;
  hipEvent_t ev_step = nullptr;
  // step tables (device + pinned host staging)
  int cap_tiles = 0;
  kstap::KParams* d_desc = nullptr;
  int32_t* d_order = nullptr;
  int64_t* d_prefix = nullptr;
  unsigned long long* d_ctr = nullptr;
  void* d_tables = nullptr;
  char* h_tables = nullptr;
  size_t tables_bytes = 0;
  // state
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Frame*> pending;
  std::vector<Frame*> active;
  std::map<uint64_t, Frame*> frames;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  std::vector<double> latencies;
  int64_t pixels_done = 0;
  double t_first = -1, t_last = -1;
  std::string fatal;

  void loop();
  void admit_locked();
  void poll_downloads_locked();
  void finish(Frame* f, stap_status st, const char* what);
};

void stap_server_s::finish(Frame* f, stap_status st, const char* what) {
  f->status = st;
  f->state = (st == STAP_OK) ? kDone : kFailed;
  f->t_done = now_s();
  if (st == STAP_OK) {
    latencies.push_back(f->t_done - f->t_submit);
    pixels_done += f->total;
    t_last = f->t_done;
  } else if (what) {
    fatal = what;
  }
  arena->release(f->off, f->bytes);
  active.erase(std::remove(active.begin(), active.end(), f), active.end());
  cv_done.notify_all();
}

// Admits waiting frames in arrival order while their buffers fit.
void stap_server_s::admit_locked() {
  while (!pending.empty() && int(active.size()) < max_inflight) {
    Frame* f = pending.front();
    size_t off = 0;
    if (!arena->alloc(f->bytes, &off)) break;
    pending.pop_front();
    f->off = off;
    active.push_back(f);
    hipError_t e = hipSuccess;
    if (!f->x_on_device)
      e = hipMemcpyAsync(arena_base + off, f->x_src, f->x_bytes, hipMemcpyHostToDevice, s_copy);
    if (e == hipSuccess && f->planes) {   // the mixed path's split, behind the upload
      const void* x = f->x_on_device ? f->x_src : static_cast<const void*>(arena_base + off);
      const stap_config& c = f->plan->cfg;
      e = hipError_t(kstap::launch_split(static_cast<const float2*>(x),
                                         reinterpret_cast<uint32_t*>(arena_base + off + f->planes_off),
                                         int64_t(c.p) * f->H * f->W * c.q, s_copy));
    }
    if (e == hipSuccess) e = hipEventRecord(f->ev_up, s_copy);
    if (e != hipSuccess) {
      finish(f, STAP_ERR_DEVICE, hipGetErrorString(e));
      continue;
    }
    f->state = kUploading;
  }
}

void stap_server_s::poll_downloads_locked() {
  std::vector<Frame*> act = active;
  for (Frame* f : act) {
    if (f->state != kDownloading) continue;
    const hipError_t e = hipEventQuery(f->ev_down);
    if (e == hipSuccess)
      finish(f, STAP_OK, nullptr);
    else if (e != hipErrorNotReady)
      finish(f, STAP_ERR_DEVICE, hipGetErrorString(e));
  }
}

void stap_server_s::loop() {
  const hipError_t de = hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  if (de != hipSuccess) {
    // the worker cannot use the device: every frame fails (none is admitted,
    // so none holds arena memory)
    fatal = hipGetErrorString(de);
    while (!(stop && pending.empty())) {
      while (!pending.empty()) {
        Frame* f = pending.front();
        pending.pop_front();
        f->status = STAP_ERR_DEVICE;
        f->state = kFailed;
        f->t_done = now_s();
      }
      cv_done.notify_all();
      cv_work.wait_for(lk, std::chrono::microseconds(200));
    }
    return;
  }
  while (true) {
    admit_locked();
    poll_downloads_locked();
    // frames whose input has arrived and that still have pixels to do
    std::vector<Frame*> ready;
    const std::vector<Frame*> act = active;   // finish() edits `active`
    for (Frame* f : act) {
      if (f->state == kUploading) {
        const hipError_t e = hipEventQuery(f->ev_up);
        if (e == hipSuccess)
          f->state = kComputing;
        else if (e != hipErrorNotReady)
          finish(f, STAP_ERR_DEVICE, hipGetErrorString(e));
      }
      if (f->state == kComputing && f->cursor < f->npos) ready.push_back(f);
    }
    if (ready.empty()) {
      if (stop && pending.empty() && active.empty()) break;
      cv_work.wait_for(lk, std::chrono::microseconds(200));
      continue;
    }
    if (int(ready.size()) > cap_tiles) ready.resize(cap_tiles);
    // fair-share slices of this step
    // slices start on a sliding-window chain
    const int64_t share = (std::max<int64_t>(16384, step_pixels / int64_t(ready.size())) + kstap::kChainNarrow - 1) /
                          kstap::kChainNarrow * kstap::kChainNarrow;
    std::vector<kstap::KParams> descs(ready.size());
    std::map<int, std::vector<int32_t>> by_cls;
    for (size_t i = 0; i < ready.size(); ++i) {
      Frame* f = ready[i];
      kstap::KParams& k = descs[i];
      const void* x = f->x_on_device ? f->x_src : static_cast<const void*>(arena_base + f->off);
      fill_params(f->plan, x, f->H, f->W, &k);
      const size_t xb = (f->x_bytes + 255) / 256 * 256;
      const size_t px = size_t(f->H) * f->W;
      if (f->planes) k.xs = reinterpret_cast<const uint32_t*>(arena_base + f->off + f->planes_off);
      k.T = reinterpret_cast<float*>(arena_base + f->off + xb);
      k.D = reinterpret_cast<uint8_t*>(arena_base + f->off + xb + (px * 4 + 255) / 256 * 256);
      k.range_first = f->cursor;
      k.range_end = std::min<int64_t>(f->npos, f->cursor + share);
      f->inflight_end = k.range_end;
      by_cls[f->cls].push_back(int32_t(i));
    }
    lk.unlock();
    // tables: descs | order | prefix (pinned staging, one copy on the compute stream)
    const int ppb = kstap::kChainNarrow;
    const size_t o_order = sizeof(kstap::KParams) * cap_tiles;
    const size_t o_prefix = o_order + sizeof(int32_t) * cap_tiles;
    std::memcpy(h_tables, descs.data(), sizeof(kstap::KParams) * descs.size());
    int32_t* h_order = reinterpret_cast<int32_t*>(h_tables + o_order);
    int64_t* h_prefix = reinterpret_cast<int64_t*>(h_tables + o_prefix);
    std::vector<std::pair<int, std::pair<size_t, size_t>>> launches;   // class, (order base, prefix base)
    size_t no = 0, np = 0;
    for (auto& kv : by_cls) {
      std::vector<int32_t>& ord = kv.second;
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return descs[a].range_end - descs[a].range_first > descs[b].range_end - descs[b].range_first;
      });
      launches.push_back({kv.first, {no, np}});
      int64_t acc = 0;
      for (int32_t t : ord) {
        h_order[no++] = t;
        h_prefix[np++] = acc;
        acc += (descs[t].range_end - descs[t].range_first + ppb - 1) / ppb;
      }
      h_prefix[np++] = acc;
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);   // else 256
    hipError_t e = hipMemcpyAsync(d_tables, h_tables, o_prefix + sizeof(int64_t) * np, hipMemcpyHostToDevice, s_comp);
    int le = (e == hipSuccess) ? kstap::launch_reset(d_ctr, int(launches.size()) * kstap::kQueues, s_comp) : int(e);
    for (size_t c = 0; c < launches.size() && le == hipSuccess; ++c) {
      const auto& L = launches[c];
      const int nt = int(by_cls[L.first].size());
      le = kstap::launch_persistent(L.first, d_desc, d_order + L.second.first, d_prefix + L.second.second, nt, ppb,
                                    d_ctr + c * kstap::kQueues, cus * 8, s_comp);
    }
    if (le == hipSuccess) le = hipEventRecord(ev_step, s_comp);
    // while the step runs: admit new frames, finish downloads
    lk.lock();
    if (le != hipSuccess) {
      for (Frame* f : ready) finish(f, STAP_ERR_DEVICE, hipGetErrorString(hipError_t(le)));
      continue;
    }
    while (true) {
      const hipError_t q = hipEventQuery(ev_step);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) {
        le = q;
        break;
      }
      admit_locked();
      poll_downloads_locked();
      cv_work.wait_for(lk, std::chrono::microseconds(100));
    }
    for (Frame* f : ready) {
      if (f->state != kComputing) continue;
      if (le != hipSuccess) {
        finish(f, STAP_ERR_DEVICE, hipGetErrorString(hipError_t(le)));
        continue;
      }
      f->cursor = f->inflight_end;
      if (f->cursor < f->npos) continue;
      const size_t xb = (f->x_bytes + 255) / 256 * 256;
      const size_t px = size_t(f->H) * f->W;
      hipError_t d = hipMemcpyAsync(f->T_out, arena_base + f->off + xb, px * 4, hipMemcpyDeviceToHost, s_copy);
      if (d == hipSuccess && f->D_out)
        d = hipMemcpyAsync(f->D_out, arena_base + f->off + xb + (px * 4 + 255) / 256 * 256, px,
                           hipMemcpyDeviceToHost, s_copy);
      if (d == hipSuccess) d = hipEventRecord(f->ev_down, s_copy);
      if (d != hipSuccess) {
        finish(f, STAP_ERR_DEVICE, hipGetErrorString(d));
        continue;
      }
      f->state = kDownloading;
    }
  }
}

extern "C" {

stap_status stap_server_create(size_t hbm_budget_bytes, int32_t max_inflight, int64_t step_pixels,
                               stap_server_t** out) {
  if (!out) return fail(STAP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < (size_t(1) << 20)) return fail(STAP_ERR_INVALID_ARG, "HBM budget below 1 MiB");
  if (max_inflight < 1 || max_inflight > 4096) return fail(STAP_ERR_INVALID_ARG, "max_inflight outside [1, 4096]");
  if (step_pixels < 0) return fail(STAP_ERR_INVALID_ARG, "step_pixels < 0");
  stap_server_s* s = new (std::nothrow) stap_server_s();
  if (!s) return fail(STAP_ERR_OUT_OF_MEMORY, "server allocation failed");
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  s->step_pixels = step_pixels > 0 ? step_pixels : (int64_t(1) << 20);
  s->cap_tiles = max_inflight;
  auto cleanup = [s]() {
    if (s->ev_step) (void)hipEventDestroy(s->ev_step);
    if (s->s_copy) (void)hipStreamDestroy(s->s_copy);
    if (s->s_comp) (void)hipStreamDestroy(s->s_comp);
    if (s->d_tables) (void)hipFree(s->d_tables);
    if (s->h_tables) (void)hipHostFree(s->h_tables);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s->arena;
    delete s;
  };
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->arena_base), hbm_budget_bytes);
  if (e != hipSuccess) {
    s->arena_base = nullptr;
    cleanup();
    return fail(STAP_ERR_OUT_OF_MEMORY, "HBM arena of %zu bytes: %s", hbm_budget_bytes, hipGetErrorString(e));
  }
  s->arena = new Arena(hbm_budget_bytes);
  const size_t o_order = sizeof(kstap::KParams) * s->cap_tiles;
  const size_t o_prefix = o_order + sizeof(int32_t) * s->cap_tiles;
  const size_t o_ctr = (o_prefix + sizeof(int64_t) * 2 * (s->cap_tiles + 1) + 255) / 256 * 256;
  s->tables_bytes = o_ctr + sizeof(unsigned long long) * (s->cap_tiles + 1) * kstap::kQueues;
  e = hipMalloc(&s->d_tables, s->tables_bytes);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->h_tables), s->tables_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_copy, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_step, hipEventDisableTiming);
  if (e != hipSuccess) {
    cleanup();
    return fail(STAP_ERR_DEVICE, "server set-up: %s", hipGetErrorString(e));
  }
  char* base = static_cast<char*>(s->d_tables);
  s->d_desc = reinterpret_cast<kstap::KParams*>(base);
  s->d_order = reinterpret_cast<int32_t*>(base + o_order);
  s->d_prefix = reinterpret_cast<int64_t*>(base + o_prefix);
  s->d_ctr = reinterpret_cast<unsigned long long*>(base + o_ctr);
  s->worker = std::thread([s]() { s->loop(); });
  *out = s;
  return ok();
}

stap_status stap_server_submit(stap_server_t* srv, const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                               int32_t x_on_device, float* T_host, uint8_t* D_host, uint64_t* ticket) {
  if (!srv || !ticket) return fail(STAP_ERR_INVALID_ARG, "server and ticket must not be NULL");
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!T_host) return fail(STAP_ERR_INVALID_ARG, "T_host is NULL");
  const stap_config& c = plan->cfg;
  const int cls = kstap::kernel_class(c.p, c.q, c.r_b, c.precision);
  if (cls < 0) return fail(STAP_ERR_UNSUPPORTED, "no kernel for p=%d q=%d r_b=%d", c.p, c.q, c.r_b);
  Frame* f = new (std::nothrow) Frame();
  if (!f) return fail(STAP_ERR_OUT_OF_MEMORY, "frame record allocation failed");
  f->plan = plan;
  f->x_src = x;
  f->x_on_device = x_on_device != 0;
  f->H = H;
  f->W = W;
  f->T_out = T_host;
  f->D_out = D_host;
  f->cls = cls;
  f->bytes = frame_bytes(plan, H, W, f->x_on_device, &f->x_bytes, &f->planes_off);
  f->planes = kstap::kernel_needs_planes(plan->cfg.p, plan->cfg.q, plan->cfg.r_b, plan->cfg.precision);
  f->total = int64_t(H) * W;
  f->npos = kstap::tiled_positions(H, W);
  if (f->bytes > srv->budget) {
    delete f;
    return fail(STAP_ERR_BUSY, "frame needs %zu bytes of device memory, the budget is %zu", size_t(f->bytes),
                srv->budget);
  }
  if (hipEventCreateWithFlags(&f->ev_up, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&f->ev_down, hipEventDisableTiming) != hipSuccess) {
    if (f->ev_up) (void)hipEventDestroy(f->ev_up);
    delete f;
    return fail(STAP_ERR_DEVICE, "event creation failed");
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) {
      (void)hipEventDestroy(f->ev_up);
      (void)hipEventDestroy(f->ev_down);
      delete f;
      return fail(STAP_ERR_INVALID_ARG, "server is shutting down");
    }
    f->ticket = srv->next_ticket++;
    f->t_submit = now_s();
    if (srv->t_first < 0) srv->t_first = f->t_submit;
    srv->frames[f->ticket] = f;
    srv->pending.push_back(f);
    *ticket = f->ticket;
  }
  srv->cv_work.notify_all();
  return ok();
}

stap_status stap_server_wait(stap_server_t* srv, uint64_t ticket, int32_t timeout_ms, double* latency_s) {
  if (!srv) return fail(STAP_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->frames.find(ticket);
  if (it == srv->frames.end()) return fail(STAP_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  Frame* f = it->second;
  auto done = [f]() { return f->state == kDone || f->state == kFailed; };
  if (timeout_ms < 0) {
    srv->cv_done.wait(lk, done);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
    return fail(STAP_ERR_BUSY, "frame %llu not finished within %d ms", (unsigned long long)ticket, timeout_ms);
  }
  const stap_status st = f->status;
  if (latency_s) *latency_s = f->t_done - f->t_submit;
  srv->frames.erase(it);
  (void)hipEventDestroy(f->ev_up);
  (void)hipEventDestroy(f->ev_down);
  delete f;
  if (st != STAP_OK) return fail(st, "frame %llu failed: %s", (unsigned long long)ticket, srv->fatal.c_str());
  return ok();
}

stap_status stap_server_stats(stap_server_t* srv, double* p50_s, double* p99_s, double* pixels_per_s,
                              int64_t* frames_done) {
  if (!srv) return fail(STAP_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  std::vector<double> l = srv->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) -> double {
    if (l.empty()) return 0.0;
    const size_t i = std::min(l.size() - 1, size_t(q * double(l.size() - 1) + 0.5));
    return l[i];
  };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (pixels_per_s) *pixels_per_s = (srv->t_last > srv->t_first) ? srv->pixels_done / (srv->t_last - srv->t_first) : 0.0;
  if (frames_done) *frames_done = int64_t(l.size());
  return ok();
}

stap_status stap_server_destroy(stap_server_t* srv) {
  if (!srv) return ok();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipStreamSynchronize(srv->s_copy);
  (void)hipStreamSynchronize(srv->s_comp);
  // teardown: failures here leave nothing to report to
  for (auto& kv : srv->frames) {
    (void)hipEventDestroy(kv.second->ev_up);
    (void)hipEventDestroy(kv.second->ev_down);
    delete kv.second;
  }
  (void)hipEventDestroy(srv->ev_step);
  (void)hipStreamDestroy(srv->s_copy);
  (void)hipStreamDestroy(srv->s_comp);
  (void)hipFree(srv->d_tables);
  (void)hipHostFree(srv->h_tables);
  (void)hipFree(srv->arena_base);
  delete srv->arena;
  delete srv;
  return ok();
}

}  // extern "C"
