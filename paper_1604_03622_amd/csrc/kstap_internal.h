// Internal interface between the host runtime (kstap_api.cpp) and the HIP
// kernels (kstap_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kstap {

constexpr int kMaxP = 8;
constexpr int kMaxQ = 32;
constexpr int kMaxN = 256;
constexpr int kMaxRA = 4;
constexpr int kMaxRB = 8;

// Everything a launch needs, passed by value as the kernel argument
// (about 1.6 KB; the kernarg segment allows 4 KB).
struct KParams {
  const float2* x;        // frame, complex64 [p][H][W][q]
  float* T;               // run: [H][W];  probe: [npix]
  uint8_t* D;             // run: [H][W] or null
  int32_t H, W;
  int32_t n, r_a, r_b;
  int32_t min_iter, max_iter;
  int32_t stat_mode;
  double eps;
  float tau;
  float bs_norm2;         // ||b_s||^2
  float h_norm2;          // ||h||^2
  int32_t r0, r1, c0, c1; // valid region, half-open
  int32_t pix_per_block;  // run: consecutive row-major pixels per workgroup
  int32_t nlogical;       // run: workgroups that carry pixels (grid is rounded up to 8)
  int64_t range_first;    // persistent: row-major pixel range [range_first, range_end) of the frame
  int64_t range_end;
  // probe
  const int32_t* pix;     // [npix][2]
  int32_t npix;
  float2* UA;             // [npix][p][r_a]
  float2* UB;             // [npix][q][r_b]
  float* eta;             // [npix]
  int32_t* iters;         // [npix]
  float2 b_s[kMaxQ];
  float2 h_s[kMaxP];
  int16_t st[2 * kMaxN];  // stencil (dr, dc)
};

enum Mode { kModeRun = 0, kModeProbe = 1 };

// Returns true if a kernel is built for (p, q, r_b bound, precision).
bool kernel_available(int p, int q, int r_b, int precision);

// Enqueues the fused per-pixel kernel.  Returns a hipError_t value.
int launch_pixels(int p, int q, int precision, int mode, const KParams& prm, hipStream_t stream);

// Kernel class id of (p, q, r_b, precision), -1 if none is built.
int kernel_class(int p, int q, int r_b, int precision);

// Enqueues the persistent batched kernel of class `cls` over the tiles
// descs[order[j]], j < nt, whose work items (runs of ppb pixels) are numbered
// by prefix[] (device arrays); counter: device work counter (must be 0).
int launch_persistent(int cls, const KParams* descs, const int32_t* order, const int64_t* prefix, int nt, int ppb,
                      unsigned long long* counter, int grid, hipStream_t stream);

// Zeroes n device counters with a kernel (no memset node in graphs).
int launch_reset(unsigned long long* counters, int n, hipStream_t stream);

// Host handles of the persistent kernel of class `cls` (arguments: descs,
// order, prefix, nt, ppb, counter) and of the counter-reset kernel
// (arguments: counters, n), for explicit graph nodes.
const void* persistent_kernel(int cls);
const void* reset_kernel();

}  // namespace kstap
