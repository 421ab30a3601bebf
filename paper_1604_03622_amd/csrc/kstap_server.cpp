// Serving: frames of mixed sizes admitted by HBM budget and processed with
// continuous batching.  See the stap_server_* declarations in kstap.h.
//
// The scheduling (arena, admission, slicing, the two-step pipeline, failure
// handling) is the device-independent core of kstap_sched.h.  This file is
// its HIP executor: one HBM arena, a copy stream for uploads, splits and
// downloads, and a compute stream that runs each step as one persistent
// launch per kernel class.  A step's tables (parameter blocks, work order,
// prefix sums, queue counters) live in one of two slots, so the next step is
// enqueued while the previous one runs and the GPU does not wait for the host
// between steps.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "kstap_host.h"
#include "kstap_internal.h"
#include "kstap_sched.h"

using namespace kstap::host;
namespace ks = kstap::sched;

namespace {

struct HipFrame {
  const stap_plan_s* plan = nullptr;
  const void* x_src = nullptr;
  bool x_on_device = false;
  int H = 0, W = 0;
  float* T_out = nullptr;
  uint8_t* D_out = nullptr;
  int cls = -1;
  bool planes = false;
  size_t x_bytes = 0, planes_off = 0;
  hipEvent_t ev_ready = nullptr;   // device-resident input: recorded on the producer's stream at submit
  hipEvent_t ev_up = nullptr, ev_down = nullptr;
};

// Device bytes of one frame: [x, unless it is already on the device] [T] [D]
// [split planes of the mixed path, if its kernel reads them].
size_t frame_bytes(const stap_plan_s* pl, int H, int W, bool x_on_device, size_t* x_bytes, size_t* planes_off) {
  const stap_config& c = pl->cfg;
  const size_t px = size_t(H) * W;
  *x_bytes = x_on_device ? 0 : px * c.p * c.q * 8;
  *planes_off = ks::Arena::round(*x_bytes) + ks::Arena::round(px * 4) + ks::Arena::round(px);
  const size_t planes = kstap::kernel_needs_planes(c.p, c.q, c.r_b, c.precision) ? px * c.p * c.q * 8 : 0;
  return *planes_off + ks::Arena::round(planes);
}

class HipExec : public ks::Exec {
 public:
  struct Slot {
    void* d_tables = nullptr;
    char* h_tables = nullptr;
    kstap::KParams* d_desc = nullptr;
    int32_t* d_order = nullptr;
    int64_t* d_prefix = nullptr;
    unsigned long long* d_ctr = nullptr;
    hipEvent_t ev = nullptr;
  };

  int device = 0, cus = 256, cap = 16;
  char* arena = nullptr;
  hipStream_t s_copy = nullptr, s_comp = nullptr;
  Slot slot[ks::Scheduler::kSlots];
  size_t o_order = 0, o_prefix = 0, o_ctr = 0, tables_bytes = 0;
  std::string err;

  hipError_t init(size_t budget, int cap_tiles) {
    cap = cap_tiles;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
      cus = 256;
    e = hipMalloc(reinterpret_cast<void**>(&arena), budget);
    if (e != hipSuccess) {
      arena = nullptr;
      return e;
    }
    o_order = sizeof(kstap::KParams) * cap;
    o_prefix = o_order + sizeof(int32_t) * cap;
    o_ctr = ks::Arena::round(o_prefix + sizeof(int64_t) * 2 * (cap + 1));
    tables_bytes = o_ctr + sizeof(unsigned long long) * (cap + 1) * kstap::kQueues;
    for (Slot& s : slot) {
      if (e == hipSuccess) e = hipMalloc(&s.d_tables, tables_bytes);
      if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s.h_tables), tables_bytes, hipHostMallocDefault);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
      if (e != hipSuccess) break;
      char* base = static_cast<char*>(s.d_tables);
      s.d_desc = reinterpret_cast<kstap::KParams*>(base);
      s.d_order = reinterpret_cast<int32_t*>(base + o_order);
      s.d_prefix = reinterpret_cast<int64_t*>(base + o_prefix);
      s.d_ctr = reinterpret_cast<unsigned long long*>(base + o_ctr);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s_copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s_comp, hipStreamNonBlocking);
    return e;
  }

  ~HipExec() override {
    // teardown: failures here leave nothing to report to
    if (s_copy) (void)hipStreamSynchronize(s_copy);
    if (s_comp) (void)hipStreamSynchronize(s_comp);
    for (Slot& s : slot) {
      if (s.ev) (void)hipEventDestroy(s.ev);
      if (s.d_tables) (void)hipFree(s.d_tables);
      if (s.h_tables) (void)hipHostFree(s.h_tables);
    }
    if (s_copy) (void)hipStreamDestroy(s_copy);
    if (s_comp) (void)hipStreamDestroy(s_comp);
    if (arena) (void)hipFree(arena);
  }

  static HipFrame* hf(ks::Frame* f) { return static_cast<HipFrame*>(f->exec); }

  bool check(hipError_t e) {
    if (e == hipSuccess) return true;
    err = hipGetErrorString(e);
    return false;
  }

  Poll poll(hipEvent_t ev) {
    const hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) return kReady;
    if (e == hipErrorNotReady) return kNotReady;
    err = hipGetErrorString(e);
    return kError;
  }

  const void* x_of(ks::Frame* f) {
    HipFrame* h = hf(f);
    return h->x_on_device ? h->x_src : static_cast<const void*>(arena + f->off);
  }

  bool upload(ks::Frame* f) override {
    HipFrame* h = hf(f);
    hipError_t e = hipSuccess;
    if (h->x_on_device && h->ev_ready) e = hipStreamWaitEvent(s_copy, h->ev_ready, 0);
    if (e == hipSuccess && !h->x_on_device)
      e = hipMemcpyAsync(arena + f->off, h->x_src, h->x_bytes, hipMemcpyHostToDevice, s_copy);
    if (e == hipSuccess && h->planes) {   // the mixed path's split, behind the upload
      const stap_config& c = h->plan->cfg;
      e = hipError_t(kstap::launch_split(static_cast<const float2*>(x_of(f)),
                                         reinterpret_cast<uint32_t*>(arena + f->off + h->planes_off),
                                         int64_t(c.p) * h->H * h->W * c.q, s_copy));
    }
    if (e == hipSuccess) e = hipEventRecord(h->ev_up, s_copy);
    return check(e);
  }
  Poll upload_state(ks::Frame* f) override { return poll(hf(f)->ev_up); }

  bool launch(int k, const std::vector<ks::Slice>& slices) override {
    Slot& s = slot[k];
    const int ppb = kstap::kChainNarrow;
    kstap::KParams* desc = reinterpret_cast<kstap::KParams*>(s.h_tables);
    int32_t* order = reinterpret_cast<int32_t*>(s.h_tables + o_order);
    int64_t* prefix = reinterpret_cast<int64_t*>(s.h_tables + o_prefix);
    std::map<int, std::vector<int32_t>> by_cls;
    for (size_t i = 0; i < slices.size(); ++i) {
      ks::Frame* f = slices[i].f;
      HipFrame* h = hf(f);
      kstap::KParams& p = desc[i];
      fill_params(h->plan, x_of(f), h->H, h->W, &p);
      const size_t xb = ks::Arena::round(h->x_bytes);
      const size_t px = size_t(h->H) * h->W;
      if (h->planes) p.xs = reinterpret_cast<const uint32_t*>(arena + f->off + h->planes_off);
      p.T = reinterpret_cast<float*>(arena + f->off + xb);
      p.D = reinterpret_cast<uint8_t*>(arena + f->off + xb + ks::Arena::round(px * 4));
      p.range_first = slices[i].first;
      p.range_end = slices[i].end;
      by_cls[h->cls].push_back(int32_t(i));
    }
    // per class: work order longest slice first, prefix sums of work items
    std::vector<std::pair<int, std::pair<size_t, size_t>>> launches;   // class, (order base, prefix base)
    size_t no = 0, np = 0;
    for (auto& kv : by_cls) {
      std::vector<int32_t>& ord = kv.second;
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return desc[a].range_end - desc[a].range_first > desc[b].range_end - desc[b].range_first;
      });
      launches.push_back({kv.first, {no, np}});
      int64_t acc = 0;
      for (int32_t t : ord) {
        order[no++] = t;
        prefix[np++] = acc;
        acc += (desc[t].range_end - desc[t].range_first + ppb - 1) / ppb;
      }
      prefix[np++] = acc;
    }
    hipError_t e = hipMemcpyAsync(s.d_tables, s.h_tables, o_prefix + sizeof(int64_t) * np, hipMemcpyHostToDevice,
                                  s_comp);
    int le = (e == hipSuccess) ? kstap::launch_reset(s.d_ctr, int(launches.size()) * kstap::kQueues, s_comp) : int(e);
    for (size_t c = 0; c < launches.size() && le == hipSuccess; ++c) {
      const auto& L = launches[c];
      const int nt = int(by_cls[L.first].size());
      le = kstap::launch_persistent(L.first, s.d_desc, s.d_order + L.second.first, s.d_prefix + L.second.second, nt,
                                    ppb, s.d_ctr + c * kstap::kQueues, cus * 8, s_comp);
    }
    if (le == hipSuccess) le = hipEventRecord(s.ev, s_comp);
    return check(hipError_t(le));
  }
  Poll step_state(int k) override { return poll(slot[k].ev); }

  bool download(ks::Frame* f) override {
    HipFrame* h = hf(f);
    const size_t xb = ks::Arena::round(h->x_bytes);
    const size_t px = size_t(h->H) * h->W;
    hipError_t e = hipMemcpyAsync(h->T_out, arena + f->off + xb, px * 4, hipMemcpyDeviceToHost, s_copy);
    if (e == hipSuccess && h->D_out)
      e = hipMemcpyAsync(h->D_out, arena + f->off + xb + ks::Arena::round(px * 4), px, hipMemcpyDeviceToHost, s_copy);
    if (e == hipSuccess) e = hipEventRecord(h->ev_down, s_copy);
    return check(e);
  }
  Poll download_state(ks::Frame* f) override { return poll(hf(f)->ev_down); }

  void drain() override {
    const hipError_t e = hipStreamSynchronize(s_comp);
    if (e != hipSuccess) err = hipGetErrorString(e);
  }

  void forget(ks::Frame* f) override {
    HipFrame* h = hf(f);
    if (!h) return;
    if (h->ev_ready) (void)hipEventDestroy(h->ev_ready);
    if (h->ev_up) (void)hipEventDestroy(h->ev_up);
    if (h->ev_down) (void)hipEventDestroy(h->ev_down);
    delete h;
    f->exec = nullptr;
  }

  std::string error() override { return err; }

  bool thread_init() override { return check(hipSetDevice(device)); }
};

}  // namespace

struct stap_server_s {
  HipExec exec;
  ks::Scheduler* sched = nullptr;
};

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
  const hipError_t e = s->exec.init(hbm_budget_bytes, max_inflight);
  if (e != hipSuccess) {
    const bool oom = s->exec.arena == nullptr;
    delete s;
    return fail(oom ? STAP_ERR_OUT_OF_MEMORY : STAP_ERR_DEVICE, "server set-up (HBM arena of %zu bytes): %s",
                hbm_budget_bytes, hipGetErrorString(e));
  }
  ks::Config cfg;
  cfg.budget = hbm_budget_bytes;
  cfg.max_inflight = max_inflight;
  cfg.max_slices = max_inflight;
  cfg.step_positions = step_pixels > 0 ? step_pixels : (int64_t(1) << 20);
  cfg.chain = kstap::kChainNarrow;   // slices start on a sliding-window chain
  s->sched = new (std::nothrow) ks::Scheduler(cfg, &s->exec);
  if (!s->sched) {
    delete s;
    return fail(STAP_ERR_OUT_OF_MEMORY, "server allocation failed");
  }
  s->sched->start();   // the worker binds the creating thread's device
  *out = s;
  return ok();
}

stap_status stap_server_submit(stap_server_t* srv, const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                               int32_t x_on_device, float* T_host, uint8_t* D_host, void* hip_stream,
                               uint64_t* ticket) {
  if (!srv || !ticket) return fail(STAP_ERR_INVALID_ARG, "server and ticket must not be NULL");
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!T_host) return fail(STAP_ERR_INVALID_ARG, "T_host is NULL");
  const stap_config& c = plan->cfg;
  if (c.filter != STAP_FILTER_KRON || c.nbank != 0 || c.passes != 1)
    return fail(STAP_ERR_UNSUPPORTED, "statistic variants (filter, bank, passes) run through stap_run_ex");
  const int cls = kstap::kernel_class(c.p, c.q, c.r_b, c.precision);
  if (cls < 0) return fail(STAP_ERR_UNSUPPORTED, "no kernel for p=%d q=%d r_b=%d", c.p, c.q, c.r_b);
  HipFrame* h = new (std::nothrow) HipFrame();
  ks::Frame* f = new (std::nothrow) ks::Frame();
  if (!h || !f) {
    delete h;
    delete f;
    return fail(STAP_ERR_OUT_OF_MEMORY, "frame record allocation failed");
  }
  h->plan = plan;
  h->x_src = x;
  h->x_on_device = x_on_device != 0;
  h->H = H;
  h->W = W;
  h->T_out = T_host;
  h->D_out = D_host;
  h->cls = cls;
  h->planes = kstap::kernel_needs_planes(c.p, c.q, c.r_b, c.precision);
  f->bytes = frame_bytes(plan, H, W, h->x_on_device, &h->x_bytes, &h->planes_off);
  f->npos = kstap::tiled_positions(H, W);
  f->pixels = int64_t(H) * W;
  f->exec = h;
  hipError_t e = hipEventCreateWithFlags(&h->ev_up, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_down, hipEventDisableTiming);
  if (e == hipSuccess && h->x_on_device) {
    // order the worker's first read of x after the work already enqueued on
    // the producer's stream
    e = hipEventCreateWithFlags(&h->ev_ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(h->ev_ready, static_cast<hipStream_t>(hip_stream));
  }
  if (e != hipSuccess) {
    srv->exec.forget(f);
    delete f;
    return fail(STAP_ERR_DEVICE, "frame events: %s", hipGetErrorString(e));
  }
  std::string err;
  st = srv->sched->submit(f, ticket, &err);
  if (st != STAP_OK) {
    srv->exec.forget(f);
    delete f;
    return fail(st, "%s", err.c_str());
  }
  return ok();
}

stap_status stap_server_wait(stap_server_t* srv, uint64_t ticket, int32_t timeout_ms, double* latency_s) {
  if (!srv) return fail(STAP_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const stap_status st = srv->sched->wait(ticket, timeout_ms, latency_s, &err);
  if (st != STAP_OK) return fail(st, "%s", err.c_str());
  return ok();
}

stap_status stap_server_stats(stap_server_t* srv, double* p50_s, double* p99_s, double* pixels_per_s,
                              int64_t* frames_done) {
  if (!srv) return fail(STAP_ERR_INVALID_ARG, "server is NULL");
  srv->sched->stats(p50_s, p99_s, pixels_per_s, frames_done);
  return ok();
}

stap_status stap_server_destroy(stap_server_t* srv) {
  if (!srv) return ok();
  srv->sched->stop();
  delete srv->sched;
  delete srv;
  return ok();
}

}  // extern "C"
