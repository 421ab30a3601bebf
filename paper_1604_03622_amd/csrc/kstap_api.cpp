// Host runtime and C ABI of the Kron-STAP library: configuration checks,
// training stencil, CFAR threshold, launch set-up.  See include/kstap.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "kstap_internal.h"

#include "kstap_host.h"
#include "kstap_tune.h"

using namespace kstap::host;

namespace {

// ------------------------------------------------------------------ batches
struct BatchClass {
  int cls = -1;                  // kernel class
  std::vector<int32_t> order;    // tiles of this class, longest first
  int ppb = 16;                  // work-item size (tiled-order positions, a multiple of the chain)
  int grid_mult = 1;             // persistent grid = compute units x 8 x grid_mult
};

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}


// Split planes of the mixed path for stap_run / stap_probe come from a
// stream-ordered pool per device that keeps its memory between calls
// (release threshold = max), so repeated runs allocate nothing new and runs
// on different streams never share a buffer.
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;

hipError_t planes_pool(hipMemPool_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pools.find(dev);
  if (it != g_pools.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  e = hipMemPoolCreate(&pool, &props);
  if (e != hipSuccess) return e;
  uint64_t keep = ~uint64_t(0);
  e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) return e;
  g_pools[dev] = pool;
  *out = pool;
  return hipSuccess;
}

// Enqueues the split of frame x into planes from the pool (k->xs); the
// caller enqueues the kernel and then planes_release on the same stream.
stap_status planes_acquire(const stap_plan_s* plan, const void* x, int H, int W, kstap::KParams* k, hipStream_t s) {
  const stap_config& c = plan->cfg;
  if (!kstap::kernel_needs_planes(c.p, c.q, c.r_b, c.precision)) return STAP_OK;
  const int64_t n = int64_t(c.p) * H * W * c.q;
  hipMemPool_t pool = nullptr;
  hipError_t e = planes_pool(&pool);
  void* xs = nullptr;
  if (e == hipSuccess) e = hipMallocFromPoolAsync(&xs, size_t(n) * 8, pool, s);
  if (e == hipErrorOutOfMemory) return fail(STAP_ERR_OUT_OF_MEMORY, "split planes: %lld bytes", (long long)(n * 8));
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "split planes: %s", hipGetErrorString(e));
  const int le = kstap::launch_split(static_cast<const float2*>(x), static_cast<uint32_t*>(xs), n, s);
  if (le != hipSuccess) {
    (void)hipFreeAsync(xs, s);   // the launch error is the one reported
    return fail(STAP_ERR_DEVICE, "split launch: %s", hipGetErrorString(hipError_t(le)));
  }
  k->xs = static_cast<const uint32_t*>(xs);
  return STAP_OK;
}

hipError_t planes_release(const kstap::KParams& k, hipStream_t s) {
  return k.xs ? hipFreeAsync(const_cast<uint32_t*>(k.xs), s) : hipSuccess;
}

// Work area of stap_run_noalloc: the split planes of the mixed path in memory
// that is reserved with the code object, so that the call allocates nothing.
// Each device that loads the library holds its own copy until the process
// ends.  In host code `scratch` only names the symbol; the device address
// comes from hipGetSymbolAddress, once per device, and only that address is
// ever handed to a kernel.
constexpr size_t kScratchBytes = size_t(STAP_NOALLOC_MAX_BYTES);
static __device__ __align__(256) uint32_t scratch[kScratchBytes / sizeof(uint32_t)];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its `scratch`

stap_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return STAP_OK;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(STAP_ERR_DEVICE, "work area address on device %d: %s", dev, hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return STAP_OK;
}

}  // namespace

struct stap_batch_s {
  std::vector<kstap::KParams> descs;
  std::vector<BatchClass> classes;
  int64_t pixels = 0;
  // device
  void* d_buf = nullptr;         // descs | order | prefix | counters
  void* d_planes = nullptr;      // split planes of the mixed-path tiles
  struct Split {
    const float2* x;
    uint32_t* xs;
    int64_t n;
  };
  std::vector<Split> splits;
  kstap::KParams* d_descs = nullptr;
  int32_t* d_order = nullptr;
  int64_t* d_prefix = nullptr;
  unsigned long long* d_counters = nullptr;
  std::vector<size_t> order_base, prefix_base;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void batch_release_graph(stap_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Numbers the work items of every class for its ppb and uploads the prefix tables.
stap_status batch_tables(stap_batch_s* b) {
  std::vector<int64_t> prefix;
  b->prefix_base.clear();
  for (const BatchClass& c : b->classes) {
    b->prefix_base.push_back(prefix.size());
    int64_t acc = 0;
    for (int32_t t : c.order) {
      prefix.push_back(acc);
      const int64_t px = b->descs[t].range_end - b->descs[t].range_first;
      acc += (px + c.ppb - 1) / c.ppb;
    }
    prefix.push_back(acc);
  }
  hipError_t e = hipMemcpy(b->d_prefix, prefix.data(), prefix.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "prefix upload: %s", hipGetErrorString(e));
  return STAP_OK;
}

// Builds the graph explicitly (no stream capture): a counter-reset kernel
// node, then one persistent kernel node per class, all depending only on the
// reset node (parallel branches).
stap_status batch_build(stap_batch_s* b) {
  batch_release_graph(b);
  stap_status st = batch_tables(b);
  if (st != STAP_OK) return st;
  const int cus = device_cus();
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "graph create: %s", hipGetErrorString(e));
  unsigned long long* ctr = b->d_counters;
  int nctr = int(b->classes.size()) * kstap::kQueues;
  void* reset_args[] = {&ctr, &nctr};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(kstap::reset_kernel());
  kp.gridDim = dim3(1);
  kp.blockDim = dim3(64);
  kp.sharedMemBytes = 0;
  kp.kernelParams = reset_args;
  kp.extra = nullptr;
  // mixed-path tiles: their split kernels run first
  std::vector<hipGraphNode_t> split_nodes;
  for (size_t i = 0; i < b->splits.size() && e == hipSuccess; ++i) {
    stap_batch_s::Split sp = b->splits[i];
    void* sargs[] = {&sp.x, &sp.xs, &sp.n};
    hipKernelNodeParams sn{};
    sn.func = const_cast<void*>(kstap::split_kernel());
    sn.gridDim = dim3(kstap::split_grid(sp.n));
    sn.blockDim = dim3(256);
    sn.kernelParams = sargs;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, nullptr, 0, &sn);
    split_nodes.push_back(node);
  }
  hipGraphNode_t reset_node = nullptr;
  if (e == hipSuccess)
    e = hipGraphAddKernelNode(&reset_node, g, split_nodes.empty() ? nullptr : split_nodes.data(), split_nodes.size(), &kp);
  for (size_t i = 0; i < b->classes.size() && e == hipSuccess; ++i) {
    const BatchClass& c = b->classes[i];
    const kstap::KParams* descs = b->d_descs;
    const int32_t* order = b->d_order + b->order_base[i];
    const int64_t* prefix = b->d_prefix + b->prefix_base[i];
    int nt = int(c.order.size());
    int ppb = c.ppb;
    unsigned long long* counter = b->d_counters + i * kstap::kQueues;
    void* args[] = {&descs, &order, &prefix, &nt, &ppb, &counter};
    hipKernelNodeParams np{};
    np.func = const_cast<void*>(kstap::persistent_kernel(c.cls));
    np.gridDim = dim3(cus * 8 * c.grid_mult);
    np.blockDim = dim3(64);
    np.sharedMemBytes = 0;
    np.kernelParams = args;
    np.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, &reset_node, 1, &np);
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(STAP_ERR_DEVICE, "graph nodes: %s", hipGetErrorString(e));
  }
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return fail(STAP_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  return STAP_OK;
}

// Work of the batch launched directly on `s` (used by the tuner, so that
// timing candidates needs no graph): the split kernels if `splits`, then the
// counter reset and the persistent kernel of class `only` (every class if -1).
stap_status batch_launch_direct(stap_batch_s* b, hipStream_t s, bool splits = true, int only = -1) {
  const int cus = device_cus();
  int le = hipSuccess;
  for (size_t i = 0; splits && i < b->splits.size() && le == hipSuccess; ++i)
    le = kstap::launch_split(b->splits[i].x, b->splits[i].xs, b->splits[i].n, s);
  if (le == hipSuccess) le = kstap::launch_reset(b->d_counters, int(b->classes.size()) * kstap::kQueues, s);
  for (size_t i = 0; i < b->classes.size() && le == hipSuccess; ++i) {
    if (only >= 0 && int(i) != only) continue;
    const BatchClass& c = b->classes[i];
    le = kstap::launch_persistent(c.cls, b->d_descs, b->d_order + b->order_base[i], b->d_prefix + b->prefix_base[i],
                                  int(c.order.size()), c.ppb, b->d_counters + i * kstap::kQueues,
                                  cus * 8 * c.grid_mult, s);
  }
  if (le != hipSuccess) return fail(STAP_ERR_DEVICE, "batch launch: %s", hipGetErrorString(hipError_t(le)));
  return STAP_OK;
}

void batch_free(stap_batch_s* b) {
  if (!b) return;
  batch_release_graph(b);
  if (b->d_buf) (void)hipFree(b->d_buf);
  if (b->d_planes) (void)hipFree(b->d_planes);
  delete b;
}

}  // namespace

extern "C" {

stap_status stap_config_default(stap_config* cfg) {
  if (!cfg) return fail(STAP_ERR_INVALID_ARG, "cfg is NULL");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->p = 3;
  cfg->q = 16;
  cfg->n = 200;
  cfg->stencil = nullptr;
  cfg->window = 0;
  cfg->guard = 3;
  cfg->r_a = 1;
  cfg->r_b = 4;
  cfg->eps = 1e-6;
  cfg->min_iter = 2;
  cfg->max_iter = 50;
  cfg->stat_mode = STAP_STAT_GLRT;
  cfg->b_steer = nullptr;
  cfg->h_steer = nullptr;
  cfg->tau = 0.0;
  cfg->pfa = 1e-4;
  cfg->precision = STAP_PREC_FP32;
  cfg->filter = STAP_FILTER_KRON;
  cfg->nbank = 0;
  cfg->passes = 1;
  return ok();
}

stap_status stap_plan_create(const stap_config* cfg, stap_plan_t** out) {
  if (!cfg || !out) return fail(STAP_ERR_INVALID_ARG, "cfg and out must not be NULL");
  *out = nullptr;
  const stap_config& c = *cfg;
  if (c.p < 1 || c.p > kstap::kMaxP) return fail(STAP_ERR_INVALID_ARG, "p = %d outside [1, %d]", c.p, kstap::kMaxP);
  if (c.q < 2 || c.q > kstap::kMaxQ) return fail(STAP_ERR_INVALID_ARG, "q = %d outside [2, %d]", c.q, kstap::kMaxQ);
  if (c.p * c.q > 128) return fail(STAP_ERR_INVALID_ARG, "p*q = %d exceeds 128", c.p * c.q);
  if (c.n < 1 || c.n > kstap::kMaxN) return fail(STAP_ERR_INVALID_ARG, "n = %d outside [1, %d]", c.n, kstap::kMaxN);
  if (c.r_a < 1 || c.r_a > std::min(c.p, kstap::kMaxRA))
    return fail(STAP_ERR_INVALID_ARG, "r_a = %d outside [1, %d]", c.r_a, std::min(c.p, kstap::kMaxRA));
  if (c.r_b < 0 || c.r_b > std::min(c.q, kstap::kMaxRB))
    return fail(STAP_ERR_INVALID_ARG, "r_b = %d outside [0, %d]", c.r_b, std::min(c.q, kstap::kMaxRB));
  if (c.min_iter < 1 || c.max_iter < c.min_iter || c.max_iter > 1000)
    return fail(STAP_ERR_INVALID_ARG, "need 1 <= min_iter <= max_iter <= 1000 (got %d, %d)", c.min_iter, c.max_iter);
  if (!std::isfinite(c.eps)) return fail(STAP_ERR_INVALID_ARG, "eps must be finite");
  if (c.stat_mode != STAP_STAT_GLRT && c.stat_mode != STAP_STAT_FIXED)
    return fail(STAP_ERR_INVALID_ARG, "unknown stat_mode %d", c.stat_mode);
  if (c.stat_mode == STAP_STAT_FIXED && !c.h_steer)
    return fail(STAP_ERR_INVALID_ARG, "STAP_STAT_FIXED needs h_steer");
  if (c.precision != STAP_PREC_FP32 && c.precision != STAP_PREC_BF16X3 && c.precision != STAP_PREC_FP32_FP64)
    return fail(STAP_ERR_INVALID_ARG, "unknown precision %d", c.precision);
  if (!(c.tau > 0.0) && !(c.pfa > 0.0 && c.pfa < 1.0))
    return fail(STAP_ERR_INVALID_ARG, "need tau > 0 or 0 < pfa < 1");
  if (!std::isfinite(c.tau)) return fail(STAP_ERR_INVALID_ARG, "tau must be finite");
  if (c.filter != STAP_FILTER_KRON && c.filter != STAP_FILTER_CLASSICAL)
    return fail(STAP_ERR_INVALID_ARG, "unknown filter %d", c.filter);
  if (c.nbank < 0 || c.nbank > 64) return fail(STAP_ERR_INVALID_ARG, "nbank = %d outside [0, 64]", c.nbank);
  if (c.passes < 1 || c.p % c.passes != 0)
    return fail(STAP_ERR_INVALID_ARG, "passes = %d must be >= 1 and divide p = %d", c.passes, c.p);
  if (c.passes > 1 && c.filter != STAP_FILTER_KRON)
    return fail(STAP_ERR_INVALID_ARG, "several passes are combined with the Kron-STAP filter only");

  stap_plan_s* pl = new (std::nothrow) stap_plan_s();
  if (!pl) return fail(STAP_ERR_OUT_OF_MEMORY, "plan allocation failed");
  pl->cfg = c;
  if (c.stencil) {
    std::set<std::pair<int, int>> seen;
    for (int m = 0; m < c.n; ++m) {
      const int dr = c.stencil[2 * m], dc = c.stencil[2 * m + 1];
      if (std::abs(dr) > 64 || std::abs(dc) > 64) {
        delete pl;
        return fail(STAP_ERR_INVALID_ARG, "stencil offset (%d, %d) beyond +-64", dr, dc);
      }
      if (dr == 0 && dc == 0) {
        delete pl;
        return fail(STAP_ERR_INVALID_ARG, "stencil contains the test pixel (0, 0)");
      }
      if (!seen.insert({dr, dc}).second) {
        delete pl;
        return fail(STAP_ERR_INVALID_ARG, "stencil offset (%d, %d) repeated", dr, dc);
      }
      pl->stencil.push_back(dr);
      pl->stencil.push_back(dc);
    }
    pl->window = 0;
  } else {
    if (c.guard < 1 || c.guard % 2 == 0) {
      delete pl;
      return fail(STAP_ERR_INVALID_ARG, "guard = %d must be odd and >= 1", c.guard);
    }
    if (c.window < 0 || (c.window > 0 && (c.window % 2 != 0 || c.window > 128))) {
      delete pl;
      return fail(STAP_ERR_INVALID_ARG, "window = %d must be 0 or even and <= 128", c.window);
    }
    int w = 0;
    if (!default_stencil(c.n, c.window, c.guard, &pl->stencil, &w)) {
      delete pl;
      return fail(STAP_ERR_INVALID_ARG, "window %d with guard %d holds fewer than n = %d offsets", c.window,
                  c.guard, c.n);
    }
    pl->window = w;
  }
  pl->dr_min = pl->dr_max = pl->stencil[0];
  pl->dc_min = pl->dc_max = pl->stencil[1];
  for (int m = 0; m < c.n; ++m) {
    pl->dr_min = std::min(pl->dr_min, pl->stencil[2 * m]);
    pl->dr_max = std::max(pl->dr_max, pl->stencil[2 * m]);
    pl->dc_min = std::min(pl->dc_min, pl->stencil[2 * m + 1]);
    pl->dc_max = std::max(pl->dc_max, pl->stencil[2 * m + 1]);
  }
  {
    // one-pixel moves right, left and down (kstap::Move): the previous pixel's
    // stencil, seen from the new pixel, is the stencil shifted by -d; o enters
    // if o is in the stencil and o + d is not, o - d leaves if o is in the
    // stencil and o - d is not
    std::set<std::pair<int, int>> st;
    for (int m = 0; m < c.n; ++m) st.insert({pl->stencil[2 * m], pl->stencil[2 * m + 1]});
    const int mvd[3][2] = {{0, 1}, {0, -1}, {1, 0}};
    bool fits = true;
    for (int mv = 0; mv < 3; ++mv) {
      for (const auto& o : st) {
        if (!st.count({o.first + mvd[mv][0], o.second + mvd[mv][1]})) {
          pl->dadd[mv].push_back(o.first);
          pl->dadd[mv].push_back(o.second);
        }
        if (!st.count({o.first - mvd[mv][0], o.second - mvd[mv][1]})) {
          pl->drem[mv].push_back(o.first - mvd[mv][0]);
          pl->drem[mv].push_back(o.second - mvd[mv][1]);
        }
      }
      fits = fits && pl->dadd[mv].size() <= 2 * size_t(kstap::kMaxDelta) &&
             pl->drem[mv].size() <= 2 * size_t(kstap::kMaxDelta);
    }
    if (!fits) {
      for (int mv = 0; mv < 3; ++mv) {
        pl->dadd[mv].clear();
        pl->drem[mv].clear();
      }
    }
  }
  pl->b_steer.assign(2 * c.q, 0.f);
  for (int j = 0; j < c.q; ++j) {
    pl->b_steer[2 * j] = c.b_steer ? c.b_steer[2 * j] : 1.f;
    pl->b_steer[2 * j + 1] = c.b_steer ? c.b_steer[2 * j + 1] : 0.f;
  }
  if (c.h_steer) pl->h_steer.assign(c.h_steer, c.h_steer + 2 * c.p);
  for (float v : pl->b_steer)
    if (!std::isfinite(v)) {
      delete pl;
      return fail(STAP_ERR_INVALID_ARG, "b_steer is not finite");
    }
  for (float v : pl->h_steer)
    if (!std::isfinite(v)) {
      delete pl;
      return fail(STAP_ERR_INVALID_ARG, "h_steer is not finite");
    }
  pl->cfg.stencil = pl->stencil.data();
  pl->cfg.b_steer = pl->b_steer.data();
  pl->cfg.h_steer = pl->h_steer.empty() ? nullptr : pl->h_steer.data();
  // null law of T under white noise with exact subspaces: Gamma(p - r_a, 1)
  // for the Kron-STAP filter, Gamma(p, 1) for the classical one
  const int dof = (c.filter == STAP_FILTER_CLASSICAL) ? c.p : c.p - c.r_a;
  if (c.tau > 0.0) {
    pl->tau = c.tau;
  } else if (dof >= 1) {
    pl->tau = gamma_isf_int(dof, c.pfa);
  } else {
    pl->tau = 0.0;   // Kron-STAP with r_a == p: F_A = 0 and T is identically 0
  }
  if (!kstap::kernel_available(c.p, c.q, c.r_b, c.precision)) {
    delete pl;
    return fail(STAP_ERR_UNSUPPORTED, "no kernel built for p=%d q=%d r_b=%d precision=%d", c.p, c.q, c.r_b,
                c.precision);
  }
  *out = pl;
  return ok();
}

stap_status stap_plan(const stap_config* cfg, stap_plan_t** out) { return stap_plan_create(cfg, out); }

stap_status stap_plan_destroy(stap_plan_t* plan) {
  delete plan;
  return ok();
}

stap_status stap_plan_info(const stap_plan_t* plan, double* tau, int32_t* window, int32_t* dr_min, int32_t* dr_max,
                           int32_t* dc_min, int32_t* dc_max) {
  if (!plan) return fail(STAP_ERR_INVALID_ARG, "plan is NULL");
  if (tau) *tau = plan->tau;
  if (window) *window = plan->window;
  if (dr_min) *dr_min = plan->dr_min;
  if (dr_max) *dr_max = plan->dr_max;
  if (dc_min) *dc_min = plan->dc_min;
  if (dc_max) *dc_max = plan->dc_max;
  return ok();
}

stap_status stap_plan_stencil(const stap_plan_t* plan, int32_t* out) {
  if (!plan || !out) return fail(STAP_ERR_INVALID_ARG, "plan and out must not be NULL");
  std::memcpy(out, plan->stencil.data(), plan->stencil.size() * sizeof(int32_t));
  return ok();
}

stap_status stap_valid_region(const stap_plan_t* plan, int32_t H, int32_t W, int32_t* r0, int32_t* r1, int32_t* c0,
                              int32_t* c1) {
  if (!plan || !r0 || !r1 || !c0 || !c1) return fail(STAP_ERR_INVALID_ARG, "NULL argument");
  if (H < 0 || W < 0) return fail(STAP_ERR_INVALID_ARG, "negative frame size");
  int a, b, cc, d;
  valid_region(plan, H, W, &a, &b, &cc, &d);
  *r0 = a;
  *r1 = b;
  *c0 = cc;
  *c1 = d;
  return ok();
}

stap_status stap_plan_order(const stap_plan_t* plan, int32_t H, int32_t W, int64_t first, int64_t count,
                            int32_t* pix, int32_t* move) {
  if (!plan || !pix) return fail(STAP_ERR_INVALID_ARG, "NULL argument");
  if (H < 1 || W < 1) return fail(STAP_ERR_INVALID_ARG, "frame %d x %d", H, W);
  const int64_t total = kstap::tiled_positions(H, W);
  if (first < 0 || count < 0 || first + count > total)
    return fail(STAP_ERR_INVALID_ARG, "positions [%lld, %lld) outside [0, %lld)", (long long)first,
                (long long)(first + count), (long long)total);
  const int chain = (plan->cfg.p * plan->cfg.q > 64) ? kstap::kChainWide : kstap::kChainNarrow;
  for (int64_t i = 0; i < count; ++i) {
    int r, c;
    const bool in = kstap::tiled_pixel(first + i, H, W, &r, &c);
    pix[2 * i] = in ? r : -1;
    pix[2 * i + 1] = in ? c : -1;
    if (move) move[i] = kstap::tiled_move(first + i, H, W, chain);
  }
  return ok();
}

stap_status stap_plan_moves(const stap_plan_t* plan, int32_t move, int32_t* nadd, int32_t* nrem, int32_t* add,
                            int32_t* rem) {
  if (!plan || !nadd || !nrem) return fail(STAP_ERR_INVALID_ARG, "NULL argument");
  if (move < 0 || move > 2) return fail(STAP_ERR_INVALID_ARG, "move %d (0 right, 1 left, 2 down)", move);
  if (plan->dadd[0].empty()) {
    *nadd = *nrem = -1;
    return ok();
  }
  *nadd = int32_t(plan->dadd[move].size() / 2);
  *nrem = int32_t(plan->drem[move].size() / 2);
  if (add) std::copy(plan->dadd[move].begin(), plan->dadd[move].end(), add);
  if (rem) std::copy(plan->drem[move].begin(), plan->drem[move].end(), rem);
  return ok();
}

stap_status stap_run(const stap_plan_t* plan, const void* x, int32_t H, int32_t W, float* T, uint8_t* D,
                     void* hip_stream) {
  stap_outputs out;
  std::memset(&out, 0, sizeof(out));
  out.T = T;
  out.D = D;
  return stap_run_ex(plan, x, H, W, &out, hip_stream);
}

stap_status stap_run_ex(const stap_plan_t* plan, const void* x, int32_t H, int32_t W, const stap_outputs* out,
                        void* hip_stream) {
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!out || !out->T) return fail(STAP_ERR_INVALID_ARG, "out and out->T must not be NULL");
  if ((out->Tpass || out->C) && plan->cfg.passes < 2)
    return fail(STAP_ERR_INVALID_ARG, "Tpass and C need a plan with passes > 1");
  kstap::KParams k;
  fill_params(plan, x, H, W, &k);
  k.T = out->T;
  k.D = out->D;
  k.E = out->E;
  k.bin = out->bin;
  k.Tpass = out->Tpass;
  k.C = out->C;
  const int64_t total = kstap::tiled_positions(H, W);
  const int64_t ppb = (plan->cfg.p * plan->cfg.q > 64) ? kstap::kChainWide : kstap::kChainNarrow;
  k.pix_per_block = int32_t(ppb);
  k.nlogical = int32_t((total + ppb - 1) / ppb);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  st = planes_acquire(plan, x, H, W, &k, s);
  if (st != STAP_OK) return st;
  const int e = kstap::launch_pixels(plan->cfg.p, plan->cfg.q, plan->cfg.precision, kstap::kModeRun, k, s);
  const hipError_t fe = planes_release(k, s);
  if (e != hipSuccess)
    return fail(STAP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  if (fe != hipSuccess) return fail(STAP_ERR_DEVICE, "split planes release: %s", hipGetErrorString(fe));
  return ok();
}

stap_status stap_lrkron(const stap_lrk_config* cfg, const void* X, float* A, float* B, double* stats,
                        void* hip_stream) {
  if (!cfg || !X || !A) return fail(STAP_ERR_INVALID_ARG, "cfg, X and A must not be NULL");
  const stap_lrk_config& c = *cfg;
  if (c.p < 1 || c.p > 8) return fail(STAP_ERR_INVALID_ARG, "p = %d outside [1, 8]", c.p);
  if (c.q < 2 || c.q > 16384) return fail(STAP_ERR_INVALID_ARG, "q = %d outside [2, 16384]", c.q);
  if (c.n < 1 || c.n * c.p > 64) return fail(STAP_ERR_INVALID_ARG, "need n >= 1 and n * p <= 64 (n = %d)", c.n);
  if (c.r_a < 1 || c.r_a > c.p) return fail(STAP_ERR_INVALID_ARG, "r_a = %d outside [1, %d]", c.r_a, c.p);
  if (c.min_iter < 1 || c.max_iter < c.min_iter || c.max_iter > 1000)
    return fail(STAP_ERR_INVALID_ARG, "need 1 <= min_iter <= max_iter <= 1000 (got %d, %d)", c.min_iter, c.max_iter);
  if (!std::isfinite(c.eps)) return fail(STAP_ERR_INVALID_ARG, "eps must be finite");
  kstap::LrkParams k;
  k.n = c.n;
  k.p = c.p;
  k.q = c.q;
  k.r_a = c.r_a;
  k.min_iter = c.min_iter;
  k.max_iter = c.max_iter;
  k.eps = c.eps;
  k.A = reinterpret_cast<float2*>(A);
  k.B = reinterpret_cast<float2*>(B);
  k.stats = stats;
  const int e = kstap::launch_lrkron(static_cast<const float2*>(X), k, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "large-q launch: %s", hipGetErrorString(hipError_t(e)));
  return ok();
}

stap_status stap_run_noalloc(const stap_plan_t* plan, const void* x, int32_t H, int32_t W, float* T, uint8_t* D,
                             void* hip_stream) {
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!T) return fail(STAP_ERR_INVALID_ARG, "T is NULL");
  const stap_config& c = plan->cfg;
  kstap::KParams k;
  fill_params(plan, x, H, W, &k);
  k.T = T;
  k.D = D;
  const int64_t total = kstap::tiled_positions(H, W);
  const int64_t ppb = (c.p * c.q > 64) ? kstap::kChainWide : kstap::kChainNarrow;
  k.pix_per_block = int32_t(ppb);
  k.nlogical = int32_t((total + ppb - 1) / ppb);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (kstap::kernel_needs_planes(c.p, c.q, c.r_b, c.precision)) {
    const int64_t n = int64_t(c.p) * H * W * c.q;
    if (size_t(n) * 8 > kScratchBytes)
      return fail(STAP_ERR_INVALID_ARG, "frame needs %lld bytes of split planes; the static work area holds %zu",
                  (long long)(n * 8), kScratchBytes);
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != STAP_OK) return st;
    const int le = kstap::launch_split(static_cast<const float2*>(x), static_cast<uint32_t*>(ws), n, s);
    if (le != hipSuccess) return fail(STAP_ERR_DEVICE, "split launch: %s", hipGetErrorString(hipError_t(le)));
    k.xs = static_cast<const uint32_t*>(ws);
  }
  const int e = kstap::launch_pixels(c.p, c.q, c.precision, kstap::kModeRun, k, s);
  if (e != hipSuccess)
    return fail(STAP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

stap_status stap_probe(const stap_plan_t* plan, const void* x, int32_t H, int32_t W, const int32_t* pix,
                       int32_t npix, const stap_probe_out* out, void* hip_stream) {
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!out || !out->T) return fail(STAP_ERR_INVALID_ARG, "out and out->T must not be NULL");
  if (plan->cfg.filter != STAP_FILTER_KRON || plan->cfg.nbank != 0 || plan->cfg.passes != 1)
    return fail(STAP_ERR_UNSUPPORTED, "the probe runs the Kron-STAP statistic of one temporal steering");
  if (npix < 0) return fail(STAP_ERR_INVALID_ARG, "npix < 0");
  if (npix == 0) return ok();
  if (!pix) return fail(STAP_ERR_INVALID_ARG, "pix is NULL");
  kstap::KParams k;
  fill_params(plan, x, H, W, &k);
  k.T = out->T;
  k.pix = pix;
  k.npix = npix;
  k.UA = reinterpret_cast<float2*>(out->UA);
  k.UB = reinterpret_cast<float2*>(out->UB);
  k.eta = out->eta;
  k.iters = out->iters;
  k.pix_per_block = 1;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  st = planes_acquire(plan, x, H, W, &k, s);
  if (st != STAP_OK) return st;
  const int e = kstap::launch_pixels(plan->cfg.p, plan->cfg.q, plan->cfg.precision, kstap::kModeProbe, k, s);
  const hipError_t fe = planes_release(k, s);
  if (e != hipSuccess)
    return fail(STAP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  if (fe != hipSuccess) return fail(STAP_ERR_DEVICE, "split planes release: %s", hipGetErrorString(fe));
  return ok();
}

stap_status stap_lrstap_probe(const stap_plan_t* plan, const stap_lrstap_config* cfg, const void* x,
                              int32_t H, int32_t W, const int32_t* pix, int32_t npix, float* T, float* U,
                              float* lam, int32_t* iters, void* hip_stream) {
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  const stap_config& c = plan->cfg;
  if (c.stat_mode != STAP_STAT_GLRT || c.nbank != 0 || c.passes != 1)
    return fail(STAP_ERR_UNSUPPORTED, "LR-STAP takes the GLRT statistic of one temporal steering and one pass");
  if (c.p * c.q > kstap::kLrsMaxPQ)
    return fail(STAP_ERR_UNSUPPORTED, "LR-STAP needs p q <= %d (got %d)", kstap::kLrsMaxPQ, c.p * c.q);
  if (npix < 0) return fail(STAP_ERR_INVALID_ARG, "npix < 0");
  if (npix == 0) return ok();
  if (!pix || !T) return fail(STAP_ERR_INVALID_ARG, "pix and T must not be NULL");
  const int r = (!cfg || cfg->r < 0) ? c.r_a * c.r_b : cfg->r;
  const int rmax = std::min(kstap::kLrsMaxR, c.p * c.q);
  if (r < 0 || r > rmax) return fail(STAP_ERR_INVALID_ARG, "LR-STAP rank %d outside [0, %d]", r, rmax);
  const int max_iter = (!cfg || cfg->max_iter == 0) ? 300 : cfg->max_iter;
  if (max_iter < 1 || max_iter > 100000) return fail(STAP_ERR_INVALID_ARG, "max_iter %d outside [1, 100000]", max_iter);
  const double tol = (!cfg || !(cfg->tol > 0.0)) ? 1e-7 : cfg->tol;
  if (!std::isfinite(tol)) return fail(STAP_ERR_INVALID_ARG, "tol must be finite");
  kstap::LrsParams k{};
  k.x = static_cast<const float2*>(x);
  k.H = H;
  k.W = W;
  k.p = c.p;
  k.q = c.q;
  k.n = c.n;
  k.r = r;
  k.max_iter = max_iter;
  k.tol = tol;
  valid_region(plan, H, W, &k.r0, &k.r1, &k.c0, &k.c1);
  double bn = 0.0;
  for (int j = 0; j < c.q; ++j) {
    k.b_s[j] = make_float2(plan->b_steer[2 * j], plan->b_steer[2 * j + 1]);
    bn += double(k.b_s[j].x) * k.b_s[j].x + double(k.b_s[j].y) * k.b_s[j].y;
  }
  k.bs_norm2 = bn;
  for (int m = 0; m < c.n; ++m) {
    k.st[2 * m] = int16_t(plan->stencil[2 * m]);
    k.st[2 * m + 1] = int16_t(plan->stencil[2 * m + 1]);
  }
  k.pix = pix;
  k.npix = npix;
  k.T = T;
  k.U = reinterpret_cast<float2*>(U);
  k.lam = lam;
  k.iters = iters;
  const int e = kstap::launch_lrstap(k, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "LR-STAP launch: %s", hipGetErrorString(hipError_t(e)));
  return ok();
}

stap_status stap_sinr_loss(const stap_true_cov* cov, const stap_filter_set* f, const float* a_grid, int32_t na,
                           const float* b_grid, int32_t nb, float* loss, void* hip_stream) {
  if (!cov || !f) return fail(STAP_ERR_INVALID_ARG, "cov and filters must not be NULL");
  const int p = cov->p, q = cov->q;
  if (p < 1 || p > 8 || q < 1 || p * q > 64) return fail(STAP_ERR_INVALID_ARG, "need 1 <= p <= 8 and p q <= 64");
  if (cov->ra < 0 || cov->ra > p || cov->rb < 0 || cov->rb > q)
    return fail(STAP_ERR_INVALID_ARG, "true factor ranks outside [0, p] x [0, q]");
  if ((cov->ra > 0 && (!cov->UA || !cov->lamA)) || (cov->rb > 0 && (!cov->UB || !cov->lamB)))
    return fail(STAP_ERR_INVALID_ARG, "true factor bases and eigenvalues must not be NULL");
  if (!(cov->sigma2 > 0.0) || !std::isfinite(cov->sigma2) || !(cov->tau2 >= 0.0) || !std::isfinite(cov->tau2))
    return fail(STAP_ERR_INVALID_ARG, "need sigma2 > 0 and tau2 >= 0");
  if (f->filter < STAP_SINR_KRON || f->filter > STAP_SINR_LRSTAP) return fail(STAP_ERR_INVALID_ARG, "unknown filter");
  if (f->npix < 0 || na < 0 || nb < 0) return fail(STAP_ERR_INVALID_ARG, "negative count");
  if (f->npix == 0 || na == 0 || nb == 0) return ok();
  if (!a_grid || !b_grid || !loss) return fail(STAP_ERR_INVALID_ARG, "a_grid, b_grid and loss must not be NULL");
  if (f->filter == STAP_SINR_LRSTAP) {
    if (f->r < 0 || f->r > p * q) return fail(STAP_ERR_INVALID_ARG, "r outside [0, p q]");
    if (f->r > 0 && !f->U) return fail(STAP_ERR_INVALID_ARG, "U must not be NULL");
  } else {
    if (f->r_a < 0 || f->r_a > p || f->r_b < 0 || f->r_b > q)
      return fail(STAP_ERR_INVALID_ARG, "r_a, r_b outside [0, p] x [0, q]");
    if ((f->r_a > 0 && !f->UA) || (f->r_b > 0 && !f->UB)) return fail(STAP_ERR_INVALID_ARG, "UA and UB must not be NULL");
  }
  kstap::SinrParams k{};
  k.kind = f->filter;
  k.p = p;
  k.q = q;
  k.npix = f->npix;
  k.r_a = f->r_a;
  k.r_b = f->r_b;
  k.r = f->r;
  k.UA = reinterpret_cast<const float2*>(f->UA);
  k.UB = reinterpret_cast<const float2*>(f->UB);
  k.U = reinterpret_cast<const float2*>(f->U);
  k.ra_t = cov->ra;
  k.rb_t = cov->rb;
  k.UA_t = reinterpret_cast<const float2*>(cov->UA);
  k.lamA_t = cov->lamA;
  k.UB_t = reinterpret_cast<const float2*>(cov->UB);
  k.lamB_t = cov->lamB;
  k.sigma2 = cov->sigma2;
  k.tau2 = cov->tau2;
  k.a_grid = reinterpret_cast<const float2*>(a_grid);
  k.b_grid = reinterpret_cast<const float2*>(b_grid);
  k.na = na;
  k.nb = nb;
  k.loss = loss;
  const int e = kstap::launch_sinr(k, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "SINR launch: %s", hipGetErrorString(hipError_t(e)));
  return ok();
}

stap_status stap_batch_create(const stap_tile* tiles, int32_t ntiles, int32_t pix_per_item, stap_batch_t** out) {
  if (!out) return fail(STAP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (ntiles < 1 || !tiles) return fail(STAP_ERR_INVALID_ARG, "need at least one tile");
  if (pix_per_item < 0 || pix_per_item > 4096) return fail(STAP_ERR_INVALID_ARG, "pix_per_item outside [0, 4096]");
  stap_batch_s* b = new (std::nothrow) stap_batch_s();
  if (!b) return fail(STAP_ERR_OUT_OF_MEMORY, "batch allocation failed");
  std::map<int, int> cls_index;
  std::vector<double> cost(ntiles);
  for (int t = 0; t < ntiles; ++t) {
    const stap_tile& tl = tiles[t];
    stap_status st = check_frame(tl.plan, tl.x, tl.H, tl.W);
    if (st != STAP_OK) {
      batch_free(b);
      return fail(st, "tile %d: %s", t, last_error().c_str());
    }
    if (!tl.T) {
      batch_free(b);
      return fail(STAP_ERR_INVALID_ARG, "tile %d: T is NULL", t);
    }
    const stap_config& c = tl.plan->cfg;
    if (c.filter != STAP_FILTER_KRON || c.nbank != 0 || c.passes != 1) {
      batch_free(b);
      return fail(STAP_ERR_UNSUPPORTED, "tile %d: statistic variants (filter, bank, passes) run through stap_run_ex",
                  t);
    }
    const int cls = kstap::kernel_class(c.p, c.q, c.r_b, c.precision);
    if (cls < 0) {
      batch_free(b);
      return fail(STAP_ERR_UNSUPPORTED, "tile %d: no kernel for p=%d q=%d r_b=%d", t, c.p, c.q, c.r_b);
    }
    kstap::KParams k;
    fill_params(tl.plan, tl.x, tl.H, tl.W, &k);
    k.T = tl.T;
    k.D = tl.D;
    k.range_first = 0;
    k.range_end = kstap::tiled_positions(tl.H, tl.W);
    b->descs.push_back(k);
    b->pixels += int64_t(tl.H) * tl.W;
    const double pq = double(c.p) * c.q;
    cost[t] = double(tl.H) * tl.W * c.n * pq * pq;
    auto it = cls_index.find(cls);
    if (it == cls_index.end()) {
      cls_index[cls] = int(b->classes.size());
      b->classes.push_back(BatchClass());
      b->classes.back().cls = cls;
      it = cls_index.find(cls);
    }
    b->classes[it->second].order.push_back(t);
  }
  // split planes of the mixed-path tiles, in one allocation
  std::vector<std::pair<int, int64_t>> need;   // tile, samples
  int64_t plane_samples = 0;
  for (int t = 0; t < ntiles; ++t) {
    const stap_config& c = tiles[t].plan->cfg;
    if (!kstap::kernel_needs_planes(c.p, c.q, c.r_b, c.precision)) continue;
    const int64_t n = int64_t(c.p) * tiles[t].H * tiles[t].W * c.q;
    need.push_back({t, n});
    plane_samples += (n + 63) / 64 * 64;
  }
  if (plane_samples > 0) {
    hipError_t pe = hipMalloc(&b->d_planes, size_t(plane_samples) * 8);
    if (pe != hipSuccess) {
      b->d_planes = nullptr;
      batch_free(b);
      return fail(STAP_ERR_OUT_OF_MEMORY, "split planes (%lld bytes): %s", (long long)(plane_samples * 8),
                  hipGetErrorString(pe));
    }
    uint32_t* at = static_cast<uint32_t*>(b->d_planes);
    for (const auto& nt : need) {
      b->descs[nt.first].xs = at;
      b->splits.push_back({static_cast<const float2*>(tiles[nt.first].x), at, nt.second});
      at += 2 * ((nt.second + 63) / 64 * 64);
    }
  }
  // work-item size and grid per class: as given, else the tuned entry of the
  // class for this device, else 16 positions and CUs x 8 workgroups
  const std::string arch = kstap::tune::device_arch();
  for (BatchClass& c : b->classes) {
    std::stable_sort(c.order.begin(), c.order.end(), [&](int32_t a, int32_t z) { return cost[a] > cost[z]; });
    if (pix_per_item > 0) {
      c.ppb = (pix_per_item + kstap::kChainNarrow - 1) / kstap::kChainNarrow * kstap::kChainNarrow;   // runs start on a chain
    } else {
      int cp, cq, crb, cprec;
      kstap::tune::Entry e;
      if (kstap::class_shape(c.cls, &cp, &cq, &crb, &cprec) && kstap::tune::lookup(arch, cp, cq, crb, cprec, &e)) {
        c.ppb = e.ppb;
        c.grid_mult = e.grid_mult;
      }
    }
  }
  // device buffer: descs | order | prefix | counters
  size_t n_order = 0, n_prefix = 0;
  for (const BatchClass& c : b->classes) {
    b->order_base.push_back(n_order);
    n_order += c.order.size();
    n_prefix += c.order.size() + 1;
  }
  const size_t o_order = sizeof(kstap::KParams) * b->descs.size();
  const size_t o_prefix = (o_order + sizeof(int32_t) * n_order + 15) / 16 * 16;
  const size_t o_ctr = (o_prefix + sizeof(int64_t) * n_prefix + 15) / 16 * 16;
  const size_t bytes = o_ctr + sizeof(unsigned long long) * b->classes.size() * kstap::kQueues;
  hipError_t e = hipMalloc(&b->d_buf, bytes);
  if (e != hipSuccess) {
    b->d_buf = nullptr;
    batch_free(b);
    return fail(STAP_ERR_OUT_OF_MEMORY, "device tile table (%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  char* base = static_cast<char*>(b->d_buf);
  b->d_descs = reinterpret_cast<kstap::KParams*>(base);
  b->d_order = reinterpret_cast<int32_t*>(base + o_order);
  b->d_prefix = reinterpret_cast<int64_t*>(base + o_prefix);
  b->d_counters = reinterpret_cast<unsigned long long*>(base + o_ctr);
  std::vector<int32_t> order;
  for (const BatchClass& c : b->classes) order.insert(order.end(), c.order.begin(), c.order.end());
  e = hipMemcpy(b->d_descs, b->descs.data(), o_order, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * n_order, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    batch_free(b);
    return fail(STAP_ERR_DEVICE, "batch set-up: %s", hipGetErrorString(e));
  }
  stap_status st = batch_build(b);
  if (st != STAP_OK) {
    std::string msg = last_error();
    batch_free(b);
    return fail(st, "%s", msg.c_str());
  }
  *out = b;
  return ok();
}

stap_status stap_batch_launch(stap_batch_t* batch, void* hip_stream) {
  if (!batch || !batch->exec) return fail(STAP_ERR_INVALID_ARG, "batch is NULL or not built");
  hipError_t e = hipGraphLaunch(batch->exec, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(STAP_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
  return ok();
}

stap_status stap_batch_tune(stap_batch_t* batch, void* hip_stream, int32_t* best_ppb, int32_t* best_grid_mult,
                            double* best_ms) {
  if (!batch) return fail(STAP_ERR_INVALID_ARG, "batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(STAP_ERR_DEVICE, "event create failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(STAP_ERR_DEVICE, "event create failed");
  }
  // per class: work items of 16..128 positions (multiples of the chain) x
  // persistent grids of 1, 2, 4 x (CUs x 8) workgroups, the class alone
  const int ppbs[] = {16, 32, 64, 128};
  const int mults[] = {1, 2, 4};
  stap_status st = batch_launch_direct(batch, s, true, int(batch->classes.size()));   // the splits only
  double total = 0.0;
  std::vector<std::pair<int, int>> best(batch->classes.size());
  std::vector<double> best_t(batch->classes.size(), 1e300);
  for (size_t i = 0; i < batch->classes.size() && st == STAP_OK; ++i) {
    BatchClass& c = batch->classes[i];
    best[i] = {c.ppb, c.grid_mult};
    for (int ppb : ppbs) {
      for (int m : mults) {
        c.ppb = ppb;
        c.grid_mult = m;
        st = batch_tables(batch);
        if (st == STAP_OK) st = batch_launch_direct(batch, s, false, int(i));   // warm-up
        hipError_t e = hipSuccess;
        float ms = 0.f;
        if (st == STAP_OK) e = hipEventRecord(e0, s);
        for (int r = 0; r < 2 && st == STAP_OK && e == hipSuccess; ++r) st = batch_launch_direct(batch, s, false, int(i));
        if (st == STAP_OK && e == hipSuccess) e = hipEventRecord(e1, s);
        if (st == STAP_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        if (st == STAP_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (st != STAP_OK) break;
        if (e != hipSuccess) {
          st = fail(STAP_ERR_DEVICE, "tuning launch: %s", hipGetErrorString(e));
          break;
        }
        if (ms / 2.0 < best_t[i]) {
          best_t[i] = ms / 2.0;
          best[i] = {ppb, m};
        }
      }
      if (st != STAP_OK) break;
    }
    c.ppb = best[i].first;
    c.grid_mult = best[i].second;
    total += best_t[i];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != STAP_OK) return st;
  hipError_t se = hipStreamSynchronize(s);
  if (se != hipSuccess) return fail(STAP_ERR_DEVICE, "tuning: %s", hipGetErrorString(se));
  st = batch_build(batch);
  if (st != STAP_OK) return st;
  const std::string arch = kstap::tune::device_arch();
  for (size_t i = 0; i < batch->classes.size(); ++i) {
    int cp, cq, crb, cprec;
    if (!kstap::class_shape(batch->classes[i].cls, &cp, &cq, &crb, &cprec)) continue;
    kstap::tune::Entry e;
    e.ppb = best[i].first;
    e.grid_mult = best[i].second;
    e.ms = best_t[i];
    std::string err;
    if (!kstap::tune::record(arch, cp, cq, crb, cprec, e, &err)) return fail(STAP_ERR_INVALID_ARG, "%s", err.c_str());
  }
  // the largest class's choice is reported (every class is in the cache)
  size_t big = 0;
  for (size_t i = 1; i < best_t.size(); ++i)
    if (best_t[i] > best_t[big]) big = i;
  if (best_ppb) *best_ppb = best.empty() ? 16 : best[big].first;
  if (best_grid_mult) *best_grid_mult = best.empty() ? 1 : best[big].second;
  if (best_ms) *best_ms = total;
  return ok();
}

stap_status stap_batch_class_info(const stap_batch_t* batch, int32_t cls, int32_t* p, int32_t* q, int32_t* rb_bound,
                                  int32_t* precision, int32_t* pix_per_item, int32_t* grid_mult) {
  if (!batch || cls < 0 || cls >= int32_t(batch->classes.size()))
    return fail(STAP_ERR_INVALID_ARG, "batch is NULL or class index out of range");
  const BatchClass& c = batch->classes[size_t(cls)];
  int cp = 0, cq = 0, crb = 0, cprec = 0;
  (void)kstap::class_shape(c.cls, &cp, &cq, &crb, &cprec);
  if (p) *p = cp;
  if (q) *q = cq;
  if (rb_bound) *rb_bound = crb;
  if (precision) *precision = cprec;
  if (pix_per_item) *pix_per_item = c.ppb;
  if (grid_mult) *grid_mult = c.grid_mult;
  return ok();
}

stap_status stap_tune_lookup(const char* arch, int32_t p, int32_t q, int32_t r_b, int32_t precision,
                             int32_t* pix_per_item, int32_t* grid_mult, int32_t* found) {
  if (!found) return fail(STAP_ERR_INVALID_ARG, "found is NULL");
  const std::string a = arch ? std::string(arch) : kstap::tune::device_arch();
  kstap::tune::Entry e;
  *found = kstap::tune::lookup(a, p, q, r_b <= 4 ? 4 : 8, precision, &e) ? 1 : 0;
  if (pix_per_item) *pix_per_item = *found ? e.ppb : 16;
  if (grid_mult) *grid_mult = *found ? e.grid_mult : 1;
  return ok();
}

stap_status stap_tune_record(const char* arch, int32_t p, int32_t q, int32_t r_b, int32_t precision,
                             int32_t pix_per_item, int32_t grid_mult, double ms) {
  if (pix_per_item < kstap::kChainNarrow || pix_per_item % kstap::kChainNarrow != 0 || pix_per_item > 4096)
    return fail(STAP_ERR_INVALID_ARG, "pix_per_item must be a multiple of %d in [%d, 4096]", kstap::kChainNarrow,
                kstap::kChainNarrow);
  if (grid_mult < 1 || grid_mult > 64) return fail(STAP_ERR_INVALID_ARG, "grid_mult outside [1, 64]");
  const std::string a = arch ? std::string(arch) : kstap::tune::device_arch();
  if (a.empty()) return fail(STAP_ERR_INVALID_ARG, "no architecture given and no device");
  kstap::tune::Entry e;
  e.ppb = pix_per_item;
  e.grid_mult = grid_mult;
  e.ms = ms;
  std::string err;
  if (!kstap::tune::record(a, p, q, r_b <= 4 ? 4 : 8, precision, e, &err)) return fail(STAP_ERR_INVALID_ARG, "%s", err.c_str());
  return ok();
}

stap_status stap_batch_info(const stap_batch_t* batch, int64_t* pixels, int32_t* classes, int32_t* pix_per_item,
                            int32_t* grid_mult) {
  if (!batch) return fail(STAP_ERR_INVALID_ARG, "batch is NULL");
  if (pixels) *pixels = batch->pixels;
  if (classes) *classes = int32_t(batch->classes.size());
  // the first class's (every class's: stap_batch_class_info)
  if (pix_per_item) *pix_per_item = batch->classes.empty() ? 16 : batch->classes[0].ppb;
  if (grid_mult) *grid_mult = batch->classes.empty() ? 1 : batch->classes[0].grid_mult;
  return ok();
}

stap_status stap_batch_destroy(stap_batch_t* batch) {
  batch_free(batch);
  return ok();
}

stap_status stap_run_batch(const stap_tile* tiles, int32_t ntiles, void* hip_stream) {
  stap_batch_t* b = nullptr;
  stap_status st = stap_batch_create(tiles, ntiles, 0, &b);
  if (st != STAP_OK) return st;
  st = stap_batch_launch(b, hip_stream);
  if (st == STAP_OK) {
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) st = fail(STAP_ERR_DEVICE, "batch execution: %s", hipGetErrorString(e));
  }
  batch_free(b);
  return st == STAP_OK ? ok() : st;
}

const char* stap_version(void) { return "kstap 0.1 (gfx950)"; }

const char* stap_last_error(void) { return last_error().c_str(); }

}  // extern "C"
