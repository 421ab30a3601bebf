// Host-side internals shared by the C ABI translation units.
#include "kstap_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <utility>

namespace kstap {
namespace host {

std::string& last_error() {
  thread_local std::string msg;
  return msg;
}



stap_status fail(stap_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  last_error() = buf;
  return st;
}

stap_status ok() {
  last_error().clear();
  return STAP_OK;
}

namespace {

// P(Gamma(k, 1) > t) = exp(-t) * sum_{i<k} t^i / i!  for integer k >= 1.
double gamma_sf_int(int k, double t) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < k; ++i) {
    term *= t / i;
    sum += term;
  }
  return std::exp(-t) * sum;
}

}  // namespace

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

// The narrow kernels (p*q <= 64) read training vectors through buffer
// records of 16 operand rows; a record starts at the window origin in the
// channel of its first row and also reaches the next channel when the 16
// rows straddle one.  Returns the record size in bytes and the smallest
// stencil offset (dr*W + dc)*q in samples.
static int64_t record_bytes(const stap_plan_s* pl, int H, int W, int64_t* st_min_out) {
  const stap_config& c = pl->cfg;
  int64_t st_min = 0, st_max = 0;
  for (int m = 0; m < c.n; ++m) {
    const int64_t o = (int64_t(pl->stencil[2 * m]) * W + pl->stencil[2 * m + 1]) * c.q;
    st_min = (m == 0 || o < st_min) ? o : st_min;
    st_max = (m == 0 || o > st_max) ? o : st_max;
  }
  // the window of the sliding-window update also reaches the vectors that leave
  for (int mv = 0; mv < 3; ++mv)
    for (size_t m = 0; 2 * m < pl->drem[mv].size(); ++m) {
      const int64_t o = (int64_t(pl->drem[mv][2 * m]) * W + pl->drem[mv][2 * m + 1]) * c.q;
      st_min = std::min(st_min, o);
      st_max = std::max(st_max, o);
    }
  const int pq = c.p * c.q;
  int span = 0;
  for (int row0 = 0; row0 < pq; row0 += 16) {
    const int last = (row0 + 15 < pq) ? row0 + 15 : pq - 1;
    span = std::max(span, last / c.q - row0 / c.q);
  }
  if (st_min_out) *st_min_out = st_min;
  return (int64_t(span) * H * W * c.q + (st_max - st_min) + c.q) * 8;
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
  k->filter = c.filter;
  k->nbank = c.nbank;
  k->passes = c.passes;
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
  int64_t st_min = 0;
  const int64_t rec = record_bytes(pl, H, W, &st_min);
  k->st_min = int32_t(st_min);
  for (int mv = 0; mv < 3; ++mv) {
    k->nadd[mv] = pl->dadd[0].empty() ? -1 : int32_t(pl->dadd[mv].size() / 2);
    k->nrem[mv] = pl->dadd[0].empty() ? -1 : int32_t(pl->drem[mv].size() / 2);
    for (size_t m = 0; m < pl->dadd[mv].size(); ++m) k->dadd[mv][m] = int16_t(pl->dadd[mv][m]);
    for (size_t m = 0; m < pl->drem[mv].size(); ++m) k->drem[mv][m] = int16_t(pl->drem[mv][m]);
  }
  k->rec_bytes = uint32_t(std::min<int64_t>(rec, (int64_t(1) << 31) - 1));   // check_frame enforces < 2^31
  return STAP_OK;
}

stap_status check_frame(const stap_plan_s* pl, const void* x, int H, int W) {
  if (!pl) return fail(STAP_ERR_INVALID_ARG, "plan is NULL");
  if (!x) return fail(STAP_ERR_INVALID_ARG, "x is NULL");
  if (H < 1 || W < 1) return fail(STAP_ERR_INVALID_ARG, "frame size %d x %d must be positive", H, W);
  const int64_t elems = int64_t(pl->cfg.p) * H * W * pl->cfg.q;
  if (elems >= (int64_t(1) << 31))
    return fail(STAP_ERR_INVALID_ARG, "frame of %lld complex samples exceeds 2^31 - 1", (long long)elems);
  const int64_t rec = record_bytes(pl, H, W, nullptr);
  if (pl->cfg.p * pl->cfg.q <= 64 && rec >= (int64_t(1) << 31))
    return fail(STAP_ERR_UNSUPPORTED, "a %d x %d channel plane at q = %d is too large: a training-vector record spans %lld bytes (limit 2^31)",
                H, W, pl->cfg.q, (long long)rec);
  return STAP_OK;
}



}  // namespace host
}  // namespace kstap
