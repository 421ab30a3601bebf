// Host runtime and C ABI of the Kron-STAP library: configuration checks,
// training stencil, CFAR threshold, launch set-up.  See include/kstap.h.
#include "../../include/kstap.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "kstap_internal.h"

struct stap_plan_s {
  stap_config cfg;                 // copy; the pointer members point into the vectors below
  std::vector<int32_t> stencil;    // n (dr, dc) pairs
  std::vector<float> b_steer;      // 2q
  std::vector<float> h_steer;      // 2p (fixed mode)
  double tau = 0.0;
  int32_t window = 0;
  int32_t dr_min = 0, dr_max = 0, dc_min = 0, dc_max = 0;
};

namespace {

thread_local std::string g_last_error;

stap_status fail(stap_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

stap_status ok() {
  g_last_error.clear();
  return STAP_OK;
}

// P(Gamma(k, 1) > t) = exp(-t) * sum_{i<k} t^i / i!  for integer k >= 1.
double gamma_sf_int(int k, double t) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < k; ++i) {
    term *= t / i;
    sum += term;
  }
  return std::exp(-t) * sum;
}

// Upper-tail quantile of Gamma(k, 1): the threshold with false-alarm rate pfa
// for a statistic whose null law (white noise, exact subspaces) is Gamma(k, 1).
double gamma_isf_int(int k, double pfa) {
  double lo = 0.0, hi = 1.0;
  while (gamma_sf_int(k, hi) > pfa) hi *= 2.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (gamma_sf_int(k, mid) > pfa)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Default training stencil: window [-W/2, W/2-1]^2 minus the centred
// guard x guard block, nearest offsets first (ties by dr, then dc).
bool default_stencil(int n, int window, int guard, std::vector<int32_t>* out, int* w_used) {
  int w = window;
  if (w <= 0) {
    w = 10;
    while (w * w - guard * guard < n) w += 2;
  }
  const int half = w / 2, g = guard / 2;
  std::vector<std::pair<int, int>> cand;
  for (int dr = -half; dr < w - half; ++dr)
    for (int dc = -half; dc < w - half; ++dc)
      if (!(std::abs(dr) <= g && std::abs(dc) <= g)) cand.emplace_back(dr, dc);
  if (int(cand.size()) < n) return false;
  std::stable_sort(cand.begin(), cand.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
    const int da = a.first * a.first + a.second * a.second, db = b.first * b.first + b.second * b.second;
    if (da != db) return da < db;
    if (a.first != b.first) return a.first < b.first;
    return a.second < b.second;
  });
  out->clear();
  for (int m = 0; m < n; ++m) {
    out->push_back(cand[m].first);
    out->push_back(cand[m].second);
  }
  *w_used = w;
  return true;
}

void valid_region(const stap_plan_s* pl, int H, int W, int* r0, int* r1, int* c0, int* c1) {
  *r0 = std::max(0, -pl->dr_min);
  *r1 = std::max(*r0, H - std::max(0, pl->dr_max));
  *c0 = std::max(0, -pl->dc_min);
  *c1 = std::max(*c0, W - std::max(0, pl->dc_max));
}

stap_status fill_params(const stap_plan_s* pl, const void* x, int H, int W, kstap::KParams* k) {
  const stap_config& c = pl->cfg;
  std::memset(k, 0, sizeof(*k));
  k->x = static_cast<const float2*>(x);
  k->H = H;
  k->W = W;
  k->n = c.n;
  k->r_a = c.r_a;
  k->r_b = c.r_b;
  k->min_iter = c.min_iter;
  k->max_iter = c.max_iter;
  k->stat_mode = c.stat_mode;
  k->eps = c.eps;
  k->tau = float(pl->tau);
  float bn = 0.f, hn = 0.f;
  for (int j = 0; j < c.q; ++j) {
    k->b_s[j] = make_float2(pl->b_steer[2 * j], pl->b_steer[2 * j + 1]);
    bn += k->b_s[j].x * k->b_s[j].x + k->b_s[j].y * k->b_s[j].y;
  }
  for (int i = 0; i < c.p && !pl->h_steer.empty(); ++i) {
    k->h_s[i] = make_float2(pl->h_steer[2 * i], pl->h_steer[2 * i + 1]);
    hn += k->h_s[i].x * k->h_s[i].x + k->h_s[i].y * k->h_s[i].y;
  }
  k->bs_norm2 = bn;
  k->h_norm2 = hn;
  for (int m = 0; m < c.n; ++m) {
    k->st[2 * m] = int16_t(pl->stencil[2 * m]);
    k->st[2 * m + 1] = int16_t(pl->stencil[2 * m + 1]);
  }
  valid_region(pl, H, W, &k->r0, &k->r1, &k->c0, &k->c1);
  return STAP_OK;
}

stap_status check_frame(const stap_plan_s* pl, const void* x, int H, int W) {
  if (!pl) return fail(STAP_ERR_INVALID_ARG, "plan is NULL");
  if (!x) return fail(STAP_ERR_INVALID_ARG, "x is NULL");
  if (H < 1 || W < 1) return fail(STAP_ERR_INVALID_ARG, "frame size %d x %d must be positive", H, W);
  const int64_t elems = int64_t(pl->cfg.p) * H * W * pl->cfg.q;
  if (elems >= (int64_t(1) << 31))
    return fail(STAP_ERR_INVALID_ARG, "frame of %lld complex samples exceeds 2^31 - 1", (long long)elems);
  return STAP_OK;
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
  if (c.precision != STAP_PREC_FP32 && c.precision != STAP_PREC_BF16X3)
    return fail(STAP_ERR_INVALID_ARG, "unknown precision %d", c.precision);
  if (!(c.tau > 0.0) && !(c.pfa > 0.0 && c.pfa < 1.0))
    return fail(STAP_ERR_INVALID_ARG, "need tau > 0 or 0 < pfa < 1");
  if (!std::isfinite(c.tau)) return fail(STAP_ERR_INVALID_ARG, "tau must be finite");

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
  if (c.tau > 0.0) {
    pl->tau = c.tau;
  } else if (c.p - c.r_a >= 1) {
    pl->tau = gamma_isf_int(c.p - c.r_a, c.pfa);
  } else {
    pl->tau = 0.0;   // r_a == p: F_A = 0 and T is identically 0
  }
  if (!kstap::kernel_available(c.p, c.q, c.r_b, c.precision)) {
    delete pl;
    return fail(STAP_ERR_UNSUPPORTED, "no kernel built for p=%d q=%d r_b=%d precision=%d", c.p, c.q, c.r_b,
                c.precision);
  }
  *out = pl;
  return ok();
}

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

stap_status stap_run(const stap_plan_t* plan, const void* x, int32_t H, int32_t W, float* T, uint8_t* D,
                     void* hip_stream) {
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!T) return fail(STAP_ERR_INVALID_ARG, "T is NULL");
  kstap::KParams k;
  fill_params(plan, x, H, W, &k);
  k.T = T;
  k.D = D;
  const int64_t total = int64_t(H) * W;
  // enough workgroups to cover 256 CUs several times over, at most 16 pixels each
  int64_t ppb = total / (256 * 8 * 4);
  ppb = std::max<int64_t>(1, std::min<int64_t>(16, ppb));
  k.pix_per_block = int32_t(ppb);
  k.nlogical = int32_t((total + ppb - 1) / ppb);
  const int e = kstap::launch_pixels(plan->cfg.p, plan->cfg.q, plan->cfg.precision, kstap::kModeRun, k,
                                     static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess)
    return fail(STAP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

stap_status stap_probe(const stap_plan_t* plan, const void* x, int32_t H, int32_t W, const int32_t* pix,
                       int32_t npix, const stap_probe_out* out, void* hip_stream) {
  stap_status st = check_frame(plan, x, H, W);
  if (st != STAP_OK) return st;
  if (!out || !out->T) return fail(STAP_ERR_INVALID_ARG, "out and out->T must not be NULL");
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
  const int e = kstap::launch_pixels(plan->cfg.p, plan->cfg.q, plan->cfg.precision, kstap::kModeProbe, k,
                                     static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess)
    return fail(STAP_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

stap_status stap_run_batch(const stap_tile* tiles, int32_t ntiles, void* hip_stream) {
  if (ntiles < 0 || (ntiles > 0 && !tiles)) return fail(STAP_ERR_INVALID_ARG, "bad tile list");
  for (int t = 0; t < ntiles; ++t) {
    stap_status st = stap_run(tiles[t].plan, tiles[t].x, tiles[t].H, tiles[t].W, tiles[t].T, tiles[t].D, hip_stream);
    if (st != STAP_OK) return st;
  }
  return ok();
}

const char* stap_version(void) { return "kstap 0.1 (gfx950)"; }

const char* stap_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
