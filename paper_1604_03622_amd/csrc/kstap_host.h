// Host-side internals shared by the C ABI translation units (plans, error
// plumbing, kernel argument set-up).  Not part of the public ABI.
#pragma once

#include <string>
#include <vector>

#include "../../include/kstap.h"
#include "kstap_internal.h"

struct stap_plan_s {
  stap_config cfg;                 // copy; the pointer members point into the vectors below
  std::vector<int32_t> stencil;    // n (dr, dc) pairs
  std::vector<float> b_steer;      // 2q
  std::vector<float> h_steer;      // 2p (fixed mode)
  double tau = 0.0;
  int32_t window = 0;
  int32_t dr_min = 0, dr_max = 0, dc_min = 0, dc_max = 0;
  // sliding-window update for a one-pixel move right, left and down
  // (kstap::Move), offsets (dr, dc) relative to the new pixel: training
  // vectors that enter (dadd) and that leave (drem); all empty when any list
  // exceeds kstap::kMaxDelta
  std::vector<int32_t> dadd[3], drem[3];
};

namespace kstap {
namespace host {

// Thread-local text returned by stap_last_error().
std::string& last_error();

// Records a formatted error message and returns `st`.
stap_status fail(stap_status st, const char* fmt, ...);

// Clears the error message and returns STAP_OK.
stap_status ok();

// Upper-tail pfa quantile of Gamma(k, 1) for integer k >= 1.
double gamma_isf_int(int k, double pfa);

// Default training stencil (window minus guard, nearest n offsets).
bool default_stencil(int n, int window, int guard, std::vector<int32_t>* out, int* w_used);

// Half-open valid region of an H x W frame.
void valid_region(const stap_plan_s* pl, int H, int W, int* r0, int* r1, int* c0, int* c1);

// Kernel arguments of one frame under a plan (outputs and ranges not set).
stap_status fill_params(const stap_plan_s* pl, const void* x, int H, int W, kstap::KParams* k);

// Argument checks shared by the frame entry points.
stap_status check_frame(const stap_plan_s* pl, const void* x, int H, int W);

}  // namespace host
}  // namespace kstap
