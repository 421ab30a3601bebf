// Kernel table and launch entry points of the fused kernels, plus the small
// helper kernels (split planes of the mixed path, counter reset).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "kstap_internal.h"

namespace kstap {

const Entry* entries_fp32(int* count);
const Entry* entries_bf16(int* count);
const Entry* entries_wide(int* count);
const Entry* entries_f32f64(int* count);

namespace {

// Frame-wide split for the mixed path: xs[i] = hi pair and xs[n + i] = lo
// pair of x[i].
__global__ __launch_bounds__(256) void split_planes(const float2* __restrict__ x, uint32_t* __restrict__ xs, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = x[i];
    const __bf16 hr = (__bf16)v.x, hi = (__bf16)v.y;
    const __bf16 lr = (__bf16)(v.x - (float)hr), li = (__bf16)(v.y - (float)hi);
    xs[i] = uint32_t(__builtin_bit_cast(uint16_t, hr)) | (uint32_t(__builtin_bit_cast(uint16_t, hi)) << 16);
    xs[n + i] = uint32_t(__builtin_bit_cast(uint16_t, lr)) | (uint32_t(__builtin_bit_cast(uint16_t, li)) << 16);
  }
}

__global__ void reset_counters(unsigned long long* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0ull;
}


// all built kernels; a kernel class is an index into this table
const std::vector<const Entry*>& table() {
  static const std::vector<const Entry*> t = [] {
    std::vector<const Entry*> v;
    for (auto part : {&entries_fp32, &entries_bf16, &entries_wide, &entries_f32f64}) {
      int n = 0;
      const Entry* e = part(&n);
      for (int i = 0; i < n; ++i) v.push_back(&e[i]);
    }
    return v;
  }();
  return t;
}

int find_index(int p, int q, int r_b, int prec) {
  const int rbm = (r_b <= 4) ? 4 : 8;
  const std::vector<const Entry*>& t = table();
  for (size_t i = 0; i < t.size(); ++i)
    if (t[i]->p == p && t[i]->q == q && t[i]->rbm == rbm && t[i]->prec == prec) return int(i);
  return -1;
}

const Entry* find(int p, int q, int r_b, int prec) {
  const int i = find_index(p, q, r_b, prec);
  return i < 0 ? nullptr : table()[i];
}

}  // namespace

bool kernel_available(int p, int q, int r_b, int precision) { return find(p, q, r_b, precision) != nullptr; }

bool kernel_needs_planes(int p, int q, int r_b, int precision) {
  const Entry* e = find(p, q, r_b, precision);
  return e && e->planes;
}

int launch_pixels(int p, int q, int precision, int mode, const KParams& prm, hipStream_t stream) {
  const Entry* e = find(p, q, prm.r_b, precision);
  if (!e) return hipErrorInvalidValue;
  return e->fn(mode, prm, stream);
}

int kernel_class(int p, int q, int r_b, int precision) {
  const int i = find_index(p, q, r_b, precision);
  return (i >= 0 && table()[i]->persist) ? i : -1;
}

int launch_persistent(int cls, const KParams* descs, const int32_t* order, const int64_t* prefix, int nt, int ppb,
                      unsigned long long* counter, int grid, hipStream_t stream) {
  if (cls < 0 || cls >= int(table().size()) || !table()[cls]->persist) return hipErrorInvalidValue;
  return table()[cls]->persist(descs, order, prefix, nt, ppb, counter, grid, stream);
}

bool class_shape(int cls, int* p, int* q, int* rbm, int* prec) {
  if (cls < 0 || cls >= int(table().size())) return false;
  const Entry* e = table()[cls];
  *p = e->p;
  *q = e->q;
  *rbm = e->rbm;
  *prec = e->prec;
  return true;
}

const void* persistent_kernel(int cls) {
  if (cls < 0 || cls >= int(table().size())) return nullptr;
  return table()[cls]->persist_fn;
}

int launch_split(const float2* x, uint32_t* xs, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_planes, dim3(split_grid(n)), dim3(256), 0, stream, x, xs, n);
  return hipGetLastError();
}

const void* split_kernel() { return reinterpret_cast<const void*>(&split_planes); }

const void* reset_kernel() { return reinterpret_cast<const void*>(&reset_counters); }

int launch_reset(unsigned long long* counters, int n, hipStream_t stream) {
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, counters, n);
  return hipGetLastError();
}

}  // namespace kstap
