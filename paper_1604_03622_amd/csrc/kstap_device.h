// Device code of the fused per-pixel Kronecker STAP kernels for gfx950
// (MI355X), shared by the translation units that instantiate them
// (kstap_kern_fp32.hip, kstap_kern_bf16.hip, kstap_kern_wide.hip).
//
// Narrow pixels (p*q <= 64): one 64-lane wavefront (one workgroup) carries
// one pixel at a time through the whole pass and walks a run of positions of
// the tiled pixel order.
//
//   a2  sample covariance S = (1/n) sum_m x_m x_m^H  (Sec. 1.1, Eq. (2)) as a
//       dense contraction on MFMA.  FP32 path: v_mfma_f32_16x16x4_f32 with
//       Re S = Xr Xr^T + Xi Xi^T and Im S = Xi Xr^T - Xr Xi^T over the upper
//       16 x 16 tiles (diagonal tiles of Im S from one product and its
//       transpose).  Mixed path: three BF16 products on pre-split planes.
//       Training vectors are read through buffer resources straight into
//       MFMA operands; workgroups that are in flight together on one XCD
//       cover a compact patch, so their windows are served from its L2.
//   a3  the rearrangement of Algorithm 1 is never materialised: block S(i,j)
//       of S is row i*p + j of R in address arithmetic only.
//   a4  A_0 = block sums of S / q^2 (Sec. 4, Eqs. (18)-(19)).
//   a5  LR-Kron (Algorithm 2) on the LDS-resident S: one sweep over S per
//       iteration computes the residual of the previous iterate, the new time
//       factor b = R^T conj(a) / ||a||^2 and the partial sums of R conj(b).
//       EIG_{r_a} (Eq. (17)): power iteration for r_a = 1, subspace
//       iteration otherwise, warm-started from the previous iterate.
//   a6  final b = R^T conj(a) / ||a||^2 and its Hermitian part are queued
//       in registers; every 64/q' pixels (q' = q rounded up to 8, 16 or 32)
//       one batched subspace iteration finds the top-r_b subspaces, q' lanes
//       per pixel with group-local DPP reductions (CGS2, residual stop).
//   a8  T = ||F_A X conj(F_B b_s)||^2 / (b_s^H F_B b_s) (Sec. 5, Eq. (25);
//       Sec. 6.3, Eq. (26)); D = T > tau.
// Wide pixels (p*q > 64): one 4-wave workgroup per pixel, see below.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kstap_internal.h"
#include "kstap_small_eig.h"

namespace kstap {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ complex
__device__ __forceinline__ float2 cz() { return make_float2(0.f, 0.f); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }
// a*b + c
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
// conj(a)*b + c
__device__ __forceinline__ float2 ccfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(-a.y, b.x, c.y)));
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return cfma(a, b, cz()); }

// double2 versions (FP64 eigensolves and normalisation of the mixed path)
template <typename C> __device__ __forceinline__ C czero();
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 ccfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) { return cfma(a, b, czero<double2>()); }
template <typename C> __device__ __forceinline__ C cto(float2 a);
template <> __device__ __forceinline__ float2 cto<float2>(float2 a) { return a; }
template <> __device__ __forceinline__ double2 cto<double2>(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ float2 tof(float2 a) { return a; }
__device__ __forceinline__ float2 tof(double2 a) { return make_float2(float(a.x), float(a.y)); }
__device__ __forceinline__ float xsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double xsqrt(double a) { return sqrt(a); }
// Scale factors that normalise an iterate or divide by a uniform norm: the
// hardware reciprocal (square root) in FP32, within one ulp, where the scale
// only has to be consistent (the next step renormalises, a statistic or a
// subspace does not depend on it); exact in FP64.  The argument is a normal
// positive number.
__device__ __forceinline__ float xrsqrt(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ double xrsqrt(double a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ float xrcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ float xmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double xmax(double a, double b) { return fmax(a, b); }

// ------------------------------------------------------- wavefront reductions
// Sum over the 64 lanes.  Four DPP steps reduce each 16-lane row (quad swaps,
// half-row mirror, row mirror: every lane then holds its row's sum), two
// row broadcasts (lane 15 -> next row, lane 31 -> rows 2 and 3) accumulate
// the rows into lane 63, and the total is read from lane 63 as a uniform
// value.  No LDS traffic.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float wsum(float v) {
  v += dpp<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp<0x141, 0xF>(v);   // row_half_mirror
  v += dpp<0x140, 0xF>(v);   // row_mirror
  v += dpp<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float2 wsum(float2 v) { return make_float2(wsum(v.x), wsum(v.y)); }
// Sums over the 64 lanes of N values at once (N a multiple of 4), each
// returned as a uniform value.  v_permlane32_swap exchanges the upper half of
// value 2m with the lower half of value 2m + 1, so one add leaves value 2m
// summed over lanes l and l + 32 in lanes 0-31 and value 2m + 1 in lanes
// 32-63; v_permlane16_swap does the same between 16-lane rows, which leaves
// four values per register, one per row (rows 0-3: values 4m, 4m + 2,
// 4m + 1, 4m + 3), and four DPP steps finish every row.  About 3.5
// instructions per value instead of the 7 of wsum.  The compiler folds the
// sum of a swap's two results into twice its first result unless the results
// pass through an empty asm first (swap_sum).
__device__ __forceinline__ float swap_sum(unsigned r0, unsigned r1) {
  asm volatile("" : "+v"(r0), "+v"(r1));
  return __builtin_bit_cast(float, r0) + __builtin_bit_cast(float, r1);
}
template <int N>
__device__ __forceinline__ void wsum_n(float (&v)[N]) {
  static_assert(N % 4 == 0, "wsum_n sums a multiple of four values");
  float w[N / 2];
#pragma unroll
  for (int m = 0; m < N / 2; ++m) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, v[2 * m]),
                                                    __builtin_bit_cast(unsigned, v[2 * m + 1]), false, false);
    w[m] = swap_sum(r[0], r[1]);
  }
#pragma unroll
  for (int m = 0; m < N / 4; ++m) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, w[2 * m]),
                                                    __builtin_bit_cast(unsigned, w[2 * m + 1]), false, false);
    float x = swap_sum(r[0], r[1]);
    x += dpp<0xB1, 0xF>(x);    // quad_perm [1,0,3,2]
    x += dpp<0x4E, 0xF>(x);    // quad_perm [2,3,0,1]
    x += dpp<0x141, 0xF>(x);   // row_half_mirror
    x += dpp<0x140, 0xF>(x);   // row_mirror: every lane holds its row's sum
    const int xi = __builtin_bit_cast(int, x);
    v[4 * m] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(xi, 0));
    v[4 * m + 2] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(xi, 16));
    v[4 * m + 1] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(xi, 32));
    v[4 * m + 3] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(xi, 48));
  }
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dppd(double v) {
  const int2 i = __builtin_bit_cast(int2, v);
  int2 o;
  o.x = __builtin_amdgcn_update_dpp(0, i.x, CTRL, ROWS, 0xF, false);
  o.y = __builtin_amdgcn_update_dpp(0, i.y, CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, o);
}
__device__ __forceinline__ double wsumd(double v) {
  v += dppd<0xB1, 0xF>(v);
  v += dppd<0x4E, 0xF>(v);
  v += dppd<0x141, 0xF>(v);
  v += dppd<0x140, 0xF>(v);
  v += dppd<0x142, 0xA>(v);
  v += dppd<0x143, 0xC>(v);
  const int2 i = __builtin_bit_cast(int2, v);
  int2 o;
  o.x = __builtin_amdgcn_readlane(i.x, 63);
  o.y = __builtin_amdgcn_readlane(i.y, 63);
  return __builtin_bit_cast(double, o);
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }   // one-wave workgroups

// LDS exchange among the lanes of one wavefront inside a workgroup of several:
// a wavefront's LDS operations are performed in issue order, so only the
// compiler has to be kept from moving accesses across this point.
__device__ __forceinline__ void lane_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <bool WAVE_LOCAL>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE_LOCAL) lane_sync();
  else wave_sync();
}

__device__ __forceinline__ float frac01(float x) { return x - floorf(x); }

// Deterministic, generic start block for subspace iteration.
__device__ __forceinline__ float2 omega(int k, int c) {
  float ph = 6.2831853f * frac01(0.6180340f * (k + 1) + 0.4142136f * (c + 1) * (k + 3));
  return make_float2(__cosf(ph), __sinf(ph));
}

// Sum over each group of QP consecutive lanes (QP = 8, 16, 32 or 64); every
// lane of a group receives its group's sum (QP = 64: a uniform value).
template <int QP>
__device__ __forceinline__ float gsum(float v) {
  if constexpr (QP == 64) {
    return wsum(v);
  } else {
    v += dpp<0xB1, 0xF>(v);
    v += dpp<0x4E, 0xF>(v);
    v += dpp<0x141, 0xF>(v);
    if constexpr (QP >= 16) v += dpp<0x140, 0xF>(v);
    if constexpr (QP == 32) v += __shfl_xor(v, 16);
    return v;
  }
}
template <int QP>
__device__ __forceinline__ float2 gsum(float2 v) { return make_float2(gsum<QP>(v.x), gsum<QP>(v.y)); }
template <int QP>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (QP == 64) {
    return wsumd(v);
  } else {
    v += dppd<0xB1, 0xF>(v);
    v += dppd<0x4E, 0xF>(v);
    v += dppd<0x141, 0xF>(v);
    if constexpr (QP >= 16) v += dppd<0x140, 0xF>(v);
    if constexpr (QP == 32) v += __shfl_xor(v, 16);
    return v;
  }
}
template <int QP>
__device__ __forceinline__ double2 gsum(double2 v) { return make_double2(gsum<QP>(v.x), gsum<QP>(v.y)); }

// ------------------------------------------------- small Hermitian subspaces
// Lanes are split into groups of QP; in each group lane k (< d) holds row k of
// a d x r block W.  Orthonormalise the columns inside every group by
// classical Gram-Schmidt with one re-orthogonalisation pass (CGS2).
template <typename S> __device__ __forceinline__ S tiny();
template <> __device__ __forceinline__ float tiny<float>() { return 1e-30f; }
template <> __device__ __forceinline__ double tiny<double>() { return 1e-280; }

template <int RM, int QP, typename C>
__device__ __forceinline__ void orth_cgs2(C (&w)[RM], int r, bool act) {
  using S = decltype(C{}.x);
#pragma unroll
  for (int c = 0; c < RM; ++c) {
    if (c >= r) continue;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      // classical GS: every projection uses the column as it entered the
      // pass (w0), applied as soon as it is known (one coefficient live)
      const C w0 = w[c];
#pragma unroll
      for (int a = 0; a < c; ++a) {
        const C h = gsum<QP>(act ? ccfma(w[a], w0, czero<C>()) : czero<C>());
        if (act) w[c] = csub(w[c], cmul(w[a], h));
      }
    }
    const S nn = gsum<QP>(act ? cabs2(w[c]) : S(0));
    const S inv = xrsqrt(xmax(nn, tiny<S>()));
    w[c] = act ? cscale(w[c], inv) : czero<C>();
  }
}

// Top-r invariant subspace of one Hermitian D x D matrix per lane group by
// subspace iteration.  Lane k of a group holds row k of the matrix (mrow) and
// row k of the orthonormal basis v (CGS2 orthonormalisation).  `cold` starts from M * Omega (Omega a
// fixed generic block), except in the groups whose lanes set `keep`, which
// take M * v instead (v a neighbouring pixel's basis, which does not pass
// the test on its own); otherwise v is the warm start of every group.  A group has converged
// when ||M V - V (V^H M V)||_F <= tol ||M V||_F for the basis entering a step;
// that step's orthonormalised M V is kept and the group's basis is frozen.
// The loop runs until every group has converged or max_steps; each group's
// result is the one it would reach alone.  sV: LDS scratch of RM * D * (64 / QP) C
// for this wavefront.  WAVE_LOCAL: the wavefront shares its workgroup with
// others that run their own solves, so it synchronises only its own lanes.
template <int RM, int QP, int D, typename C, bool WAVE_LOCAL = false>
__device__ __forceinline__ int group_subspace(const float2 (&mrow)[D], bool row_ok, int r, C (&v)[RM],
                                              C* sV, bool cold, int max_steps, double tol, bool keep = false) {
  using S = decltype(C{}.x);
  constexpr int G = 64 / QP;
  const int lane = threadIdx.x & 63, g = lane / QP, k = lane % QP;   // lane within its wavefront
  if (cold) {
    // FP64 solves: recompute the start block on every call (an empty asm
    // makes the row index opaque); hoisted out of the pixel loop, its
    // widened values would be spilled and reloaded instead
    int kk = k;
    if constexpr (sizeof(S) == 8) asm volatile("" : "+v"(kk));
#pragma unroll
    for (int c = 0; c < RM; ++c)
      if (!keep) v[c] = (row_ok && c < r) ? cto<C>(omega(kk, c)) : czero<C>();
  }
  // a start block (Omega, or a kept v) is not tested on the first step
  bool tested = !cold;
  bool done = false;
  int step = 0;
  while (true) {
    if (row_ok) {
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < r) sV[(c * D + k) * G + g] = v[c];
    }
    lds_sync<WAVE_LOCAL>();
    C w[RM];
#pragma unroll
    for (int c = 0; c < RM; ++c) w[c] = czero<C>();
    if (row_ok) {
#pragma unroll
      for (int l = 0; l < D; ++l) {
        float2 m = mrow[l];
        // keep the widening of the matrix row inside the loop (an empty asm
        // makes the value opaque), so it is not hoisted into extra registers
        asm volatile("" : "+v"(m.x), "+v"(m.y));
        const C mc = cto<C>(m);
#pragma unroll
        for (int c = 0; c < RM; ++c)
          if (c < r) w[c] = cfma(mc, sV[(c * D + l) * G + g], w[c]);
      }
    }
    lds_sync<WAVE_LOCAL>();
    bool conv = false;
    if (tested) {
      // residual W - V (V^H W), one column at a time
      S rn = 0, wn = 0;
#pragma unroll
      for (int b = 0; b < RM; ++b) {
        if (b >= r) continue;
        C rr = w[b];
#pragma unroll
        for (int a = 0; a < RM; ++a) {
          if (a >= r) continue;
          const C hb = gsum<QP>(row_ok ? ccfma(v[a], w[b], czero<C>()) : czero<C>());
          rr = csub(rr, cmul(v[a], hb));
        }
        if (row_ok) {
          rn += cabs2(rr);
          wn += cabs2(w[b]);
        }
      }
      rn = gsum<QP>(rn);
      wn = gsum<QP>(wn);
      conv = rn <= S(tol * tol) * wn;
    }
    orth_cgs2<RM, QP, C>(w, r, row_ok);
    // a group keeps the first basis computed from a converged one and is
    // frozen from then on, so its result does not depend on its neighbours
    if (!done) {
#pragma unroll
      for (int c = 0; c < RM; ++c) v[c] = w[c];
    }
    done = done || conv;
    tested = true;
    ++step;
    if (__ballot(!done) == 0 || step >= max_steps) break;
  }
  return step;
}

// Top-r invariant subspace of a small Hermitian P x P matrix (the factor A),
// computed identically by every lane with no cross-lane traffic: the
// subspace iteration, CGS2 and stopping rule of group_subspace, on a matrix
// read through M(i, j).  V[c][i] is entry i of basis column c; `cold` starts
// from M * Omega, otherwise V is the warm start.  Returns the step count.
template <int RM, int P, typename C, typename MF>
__device__ __forceinline__ int uniform_subspace(MF M, int r, C (&V)[RM][P], bool cold, int max_steps, double tol) {
  using S = decltype(C{}.x);
  if (cold) {
#pragma unroll
    for (int c = 0; c < RM; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i) V[c][i] = (c < r) ? cto<C>(omega(i, c)) : czero<C>();
  }
  bool tested = !cold;
  bool done = false;
  int step = 0;
  while (true) {
    C Wm[RM][P];
#pragma unroll
    for (int c = 0; c < RM; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i) {
        C sacc = czero<C>();
        if (c < r) {
#pragma unroll
          for (int j = 0; j < P; ++j) sacc = cfma(M(i, j), V[c][j], sacc);
        }
        Wm[c][i] = sacc;
      }
    bool conv = false;
    if (tested) {
      // residual W - V (V^H W)
      S rn = 0, wn = 0;
#pragma unroll
      for (int b = 0; b < RM; ++b) {
        if (b >= r) continue;
        C hb[RM];
#pragma unroll
        for (int a = 0; a < RM; ++a) {
          C d = czero<C>();
          if (a < r) {
#pragma unroll
            for (int i = 0; i < P; ++i) d = ccfma(V[a][i], Wm[b][i], d);
          }
          hb[a] = d;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) {
          C rr = Wm[b][i];
#pragma unroll
          for (int a = 0; a < RM; ++a)
            if (a < r) rr = csub(rr, cmul(V[a][i], hb[a]));
          rn += cabs2(rr);
          wn += cabs2(Wm[b][i]);
        }
      }
      conv = rn <= S(tol * tol) * wn;
    }
    // CGS2 on the columns of W
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      if (c >= r) continue;
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        C h[RM];
#pragma unroll
        for (int a = 0; a < RM; ++a) {
          C d = czero<C>();
          if (a < c) {
#pragma unroll
            for (int i = 0; i < P; ++i) d = ccfma(Wm[a][i], Wm[c][i], d);
          }
          h[a] = d;
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
          for (int a = 0; a < RM; ++a)
            if (a < c) Wm[c][i] = csub(Wm[c][i], cmul(Wm[a][i], h[a]));
      }
      S nn = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) nn += cabs2(Wm[c][i]);
      const S inv = xrsqrt(xmax(nn, tiny<S>()));
#pragma unroll
      for (int i = 0; i < P; ++i) Wm[c][i] = cscale(Wm[c][i], inv);
    }
    // as in group_subspace: keep the first basis computed from a converged one
    if (!done) {
#pragma unroll
      for (int c = 0; c < RM; ++c)
#pragma unroll
        for (int i = 0; i < P; ++i) V[c][i] = Wm[c][i];
    }
    done = done || conv;
    tested = true;
    ++step;
    if (done || step >= max_steps) break;
  }
  return step;
}

// Dominant eigenvector of a Hermitian P x P matrix, the same for every lane;
// M(i, j) returns its entries (registers or LDS).  Power iteration; stop on
// ||M u - (u^H M u) u|| <= tol ||M u||.
template <int P, typename C, typename MF>
__device__ __forceinline__ void power_top(MF M, C (&u)[P], bool cold, int max_steps, double tol) {
  using S = decltype(C{}.x);
  if (cold) {
    int jb = 0;
    S db = M(0, 0).x;
#pragma unroll
    for (int j = 1; j < P; ++j)
      if (M(j, j).x > db) {
        db = M(j, j).x;
        jb = j;
      }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      C s = czero<C>();
#pragma unroll
      for (int j = 0; j < P; ++j) s = (j == jb) ? M(i, j) : s;
      u[i] = s;
    }
    S nn = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) nn += cabs2(u[i]);
    const S inv = nn > S(0) ? xrsqrt(xmax(nn, tiny<S>())) : S(0);
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = cscale(u[i], inv);
  }
  for (int step = 0; step < max_steps; ++step) {
    C w[P];
    S lam = 0, wn = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      C s = czero<C>();
#pragma unroll
      for (int j = 0; j < P; ++j) s = cfma(M(i, j), u[j], s);
      w[i] = s;
      lam += u[i].x * s.x + u[i].y * s.y;
      wn += cabs2(s);
    }
    S rn = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) rn += cabs2(csub(w[i], cscale(u[i], lam)));
    if (!(wn > S(0))) break;
    const S inv = xrsqrt(xmax(wn, tiny<S>()));
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = cscale(w[i], inv);
    if (rn <= S(tol * tol) * wn) break;
  }
}

// Training-vector load.  Lanes whose element does not exist (rows past p*q,
// vectors past n) read a zero from kZeroVec instead of taking a branch, so
// every load is issued unconditionally and its value is used as loaded.
// Without branches around the loads the compiler counts the loads in flight
// exactly and waits only for the ones an MFMA is about to consume, which
// keeps the prefetch ring full.
__device__ float2 kZeroVec[1];   // never written
__device__ __forceinline__ float2 load_or_zero(const float2* p, bool keep) {
  const float2* a = keep ? p : kZeroVec;
  return *a;
}

// Training vectors of the narrow kernels are read through buffer resources:
// one record per 16-row operand block, based at the pixel's window origin in
// the channel of the block's first row.  A lane's load offset is its row
// offset (loff) plus the stencil entry's byte offset (sOffB, in LDS).  Rows
// past p*q and entries past n carry kOut, which lies beyond every record, so
// the hardware returns zeros for them: no branch, select or 64-bit address
// arithmetic per load.
constexpr uint32_t kOut = 0x80000000u;
constexpr int kOffPad = 64;   // sOffB entries past kMaxN (prefetch overrun, all kOut)

template <int Q>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const float2* xwin, int64_t plane, uint32_t rec, int I) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(xwin + int64_t((16 * I) / Q) * plane), (short)0, int(rec),
                                           0x00020000);
}
__device__ __forceinline__ float2 bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Narrow kernels keep S in LDS as its upper q x q blocks S(i, j), i <= j, with
// a padded row stride q + 1 (the lower blocks are their conjugate
// transposes); block (i, j) starts at sblk(i, j).
template <int P, int Q>
__device__ __forceinline__ int sblk(int i, int j) {
  return (i * P - i * (i - 1) / 2 + (j - i)) * Q * (Q + 1);
}
template <int P, int Q>
__device__ __forceinline__ float2 sget(const float2* sS, int i, int j, int k, int l) {
  if (i <= j) return sS[sblk<P, Q>(i, j) + k * (Q + 1) + l];
  const float2 v = sS[sblk<P, Q>(j, i) + l * (Q + 1) + k];
  return make_float2(v.x, -v.y);
}
// Stores element (a, b), a <= b, of the stacked pq x pq matrix (and, inside a
// diagonal block, its mirror).  Only elements with a <= b are written, so
// every position has exactly one writer.
template <int P, int Q>
__device__ __forceinline__ void sput(float2* sS, int a, int b, float2 v) {
  const int ba = a / Q, ka = a - ba * Q, bb = b / Q, kb = b - bb * Q;
  sS[sblk<P, Q>(ba, bb) + ka * (Q + 1) + kb] = v;
  if (ba == bb) sS[sblk<P, Q>(ba, bb) + kb * (Q + 1) + ka] = make_float2(v.x, -v.y);
}

// Block sums of S and the lane's part of ||S||_F^2, gathered while S is
// stored (for q a multiple of 16, where every 16 x 16 tile lies in one q x q
// block): a0[i*P + j] = sum_kl S(i,j)_kl for i <= j (a lower block's sum is
// the conjugate), each element counted with its mirror.
template <int P>
struct SSums {
  float2 a0[P * P];
  float nr;
};
// off: the element is not on the diagonal of S.
template <int P, int Q>
__device__ __forceinline__ void ssums_add(SSums<P>& ss, int I, int J, bool off, float2 v) {
  if constexpr (Q % 16 == 0) {
    const int bi = (16 * I) / Q, bj = (16 * J) / Q;   // constants once the tile loops unroll
    const float m = cabs2(v);
    if (bi != bj) {
      ss.a0[bi * P + bj] = cadd(ss.a0[bi * P + bj], v);
      ss.nr += 2.f * m;
    } else if (off) {
      ss.a0[bi * P + bi].x += 2.f * v.x;   // v + conj(v)
      ss.nr += 2.f * m;
    } else {
      ss.a0[bi * P + bi] = cadd(ss.a0[bi * P + bi], v);
      ss.nr += m;
    }
  }
}

// Element (tr, tc) of the 16 x 16 MFMA tile (I, J), I <= J: row 16 I + tr,
// column 16 J + tc of the stacked matrix, 0 <= tr, tc < 16.  Written so that
// what the tile indices fix (the tile lies inside the matrix, above its
// diagonal, inside one q x q block) folds once the tile loops unroll: only
// diagonal and ragged tiles test their lanes, and no per-lane predicate of
// an off-diagonal tile is kept live across the pixel loop.
template <int P, int Q>
__device__ __forceinline__ bool tile_in(int I, int J, int tr, int tc) {
  constexpr int PQ = P * Q;
  return (16 * I + 16 <= PQ || 16 * I + tr < PQ) && (16 * J + 16 <= PQ || 16 * J + tc < PQ);
}
// inside the matrix and on or above its diagonal (row == col iff I == J and
// tr == tc, since |tc - tr| < 16)
template <int P, int Q>
__device__ __forceinline__ bool tile_keep(int I, int J, int tr, int tc) {
  return tile_in<P, Q>(I, J, tr, tc) && (J > I || tr <= tc);
}
template <int P, int Q>
__device__ __forceinline__ float2 tile_get(const float2* sS, int I, int J, int tr, int tc) {
  if constexpr (Q % 16 == 0) {   // the tile lies in upper block ((16 I) / q, (16 J) / q)
    return sS[sblk<P, Q>((16 * I) / Q, (16 * J) / Q) + ((16 * I) % Q + tr) * (Q + 1) + (16 * J) % Q + tc];
  } else {
    const int row = 16 * I + tr, col = 16 * J + tc;
    return sget<P, Q>(sS, row / Q, col / Q, row % Q, col % Q);
  }
}
// sput of a tile element that tile_keep accepts
template <int P, int Q>
__device__ __forceinline__ void tile_put(float2* sS, int I, int J, int tr, int tc, float2 v) {
  if constexpr (Q % 16 == 0) {
    const int bi = (16 * I) / Q, bj = (16 * J) / Q;
    const int ka = (16 * I) % Q + tr, kb = (16 * J) % Q + tc;
    sS[sblk<P, Q>(bi, bj) + ka * (Q + 1) + kb] = v;
    if (bi == bj) sS[sblk<P, Q>(bi, bj) + kb * (Q + 1) + ka] = make_float2(v.x, -v.y);
  } else {
    sput<P, Q>(sS, 16 * I + tr, 16 * J + tc, v);
  }
}

// ------------------------------------------------------------ a2, FP32
// Classes where the tile row and column are made opaque, so that the S
// element addresses and the diagonal tiles' lane masks are formed where used,
// per pixel, instead of being hoisted out of the pixel loop, spilled and
// reloaded: q a multiple of 16 (one base address per lane, the tile offsets
// are constants), and the classes whose addresses do not fit in registers
// beside the rest of the pixel state.
template <int P, int Q>
constexpr bool kOpaqueStore = Q % 16 == 0 || (P == 3 && Q == 12) || (P == 4 && Q == 8) || (P == 6 && Q == 8);

// S = (1/n) sum_m x_m x_m^H of one pixel on v_mfma_f32_16x16x4_f32, written
// to LDS as the full Hermitian pq x pq matrix (row-major).
template <int P, int Q>
__device__ __forceinline__ void scm_fp32(const float2* xwin, int64_t plane, uint32_t rec, const uint32_t* sOffB,
                                         const uint32_t (&loff)[(P * Q + 15) / 16], int n, float2* sS,
                                         float* sP, SSums<P>& ss) {
  constexpr int PQ = P * Q;
  constexpr int NB = (PQ + 15) / 16;
  constexpr int NT = NB * (NB + 1) / 2;
  constexpr int NO = NB * (NB - 1) / 2;
  const int lane = threadIdx.x;
    f4 accR[NT], accI[NO > 0 ? NO : 1], accD[NB];
#pragma unroll
    for (int t = 0; t < NT; ++t) accR[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < (NO > 0 ? NO : 1); ++t) accI[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NB; ++t) accD[t] = f4{0.f, 0.f, 0.f, 0.f};

    const int nch = (n + 3) >> 2;
    // operand ring: chunk ch lives in slot ch % PF; PF - 1 chunks in flight
    constexpr int PF = 4;
    float2 ring[PF][NB];
    __amdgpu_buffer_rsrc_t rs[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) rs[I] = block_rsrc<Q>(xwin, plane, rec, I);
    auto fetch = [&](int ch, float2 (&v)[NB]) {
      const uint32_t off = sOffB[ch * 4 + (lane >> 4)];
#pragma unroll
      for (int I = 0; I < NB; ++I) v[I] = bload(rs[I], loff[I] + off);
    };
    // MFMAs of one 4-vector chunk
    auto accumulate = [&](const float2 (&v)[NB]) {
      float xr[NB], xi[NB], nxr[NB];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        xr[I] = v[I].x;
        xi[I] = v[I].y;
        nxr[I] = -v[I].x;
      }
      // first product of every accumulator, then the second: no two
      // consecutive MFMAs write the same accumulator
      {
        int t = 0, u = 0;
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = I; J < NB; ++J) {
            accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[I], xr[J], accR[t], 0, 0, 0);
            if (J > I) {
              accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[I], xr[J], accI[u], 0, 0, 0);
              ++u;
            } else {
              accD[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[I], xr[I], accD[I], 0, 0, 0);
            }
            ++t;
          }
      }
      {
        int t = 0, u = 0;
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = I; J < NB; ++J) {
            accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[I], xi[J], accR[t], 0, 0, 0);
            if (J > I) {
              accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(nxr[I], xi[J], accI[u], 0, 0, 0);
              ++u;
            }
            ++t;
          }
      }
    };
#pragma unroll
    for (int s0 = 0; s0 < PF - 1; ++s0) {   // in order: oldest chunk's loads first
      __builtin_amdgcn_sched_barrier(0);
      fetch(s0, ring[s0]);
    }
    // whole groups of PF chunks: branch-free, so the loads of the ring are
    // waited for one chunk at a time (fetches past n read zeros)
    int ch0 = 0;
    for (; ch0 + PF <= nch; ch0 += PF) {
#pragma unroll
      for (int sl = 0; sl < PF; ++sl) {
        // keep each chunk's instructions in place: hoisting work on a slot
        // that was just fetched would wait for its load right away
        __builtin_amdgcn_sched_barrier(0);
        fetch(ch0 + sl + PF - 1, ring[(sl + PF - 1) % PF]);
        accumulate(ring[sl]);
      }
    }
    // the last nch - ch0 < PF chunks are already in ring slots 0, 1, ...
#pragma unroll
    for (int sl = 0; sl < PF - 1; ++sl)
      if (ch0 + sl < nch) accumulate(ring[sl]);

    // S to LDS (upper blocks), scaled by 1/n.  MFMA output layout: lane l,
    // register q holds row 4*(l/16) + q, column l % 16 of the 16 x 16 tile.
    // Im of a diagonal tile is P - P^T with P = Xi Xr^T: the raw P goes through
    // the scratch sP ([NB][16][16]) for the transposed element.
    const float inv_n = 1.f / float(n);
    int trow = 4 * (lane >> 4), tcol = lane & 15;
    if constexpr (kOpaqueStore<P, Q>) asm volatile("" : "+v"(trow), "+v"(tcol));
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) sP[(I * 16 + trow + q4) * 16 + tcol] = accD[I][q4];
    wave_sync();
    {
      int t = 0, u = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int J = I; J < NB; ++J) {
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            const int tr = trow + q4;
            if (tile_keep<P, Q>(I, J, tr, tcol)) {
              const float re = accR[t][q4] * inv_n;
              const float im = (J > I) ? accI[u][q4] * inv_n
                                       : (accD[I][q4] - sP[(I * 16 + tcol) * 16 + tr]) * inv_n;
              tile_put<P, Q>(sS, I, J, tr, tcol, make_float2(re, im));
              ssums_add<P, Q>(ss, I, J, I != J || tr != tcol, make_float2(re, im));
            }
          }
          if (J > I) ++u;
          ++t;
        }
      }
    }
    wave_sync();
}

// Sliding-window update of S (FP32): from the previous pixel's S (in LDS),
// n S += sum over entering vectors x x^H - sum over leaving ones.  sAdd /
// sRem: byte offsets (kOut past nadd / nrem and for 8 entries beyond).
// Up to three 16-row blocks (where registers allow a third accumulator per
// tile), every tile takes three real products per chunk instead of four:
// with P1 = Xr Xr^T, P2 = Xi Xi^T and P3 = (Xr + Xi)(Xr - Xi)^T, Re S =
// P1 + P2 and Im S = P3 - P1 + P2, and the diagonal of S is stored real.
// Larger classes take Re and Im of every tile with two products each (no
// transpose through LDS).
template <int P, int Q>
__device__ __forceinline__ void scm_fp32_delta(const float2* xwin, int64_t plane, uint32_t rec,
                                               const uint32_t* sAdd, int nadd, const uint32_t* sRem, int nrem,
                                               const uint32_t (&loff)[(P * Q + 15) / 16], int n, float2* sS,
                                               SSums<P>& ss) {
  constexpr int PQ = P * Q;
  constexpr int NB = (PQ + 15) / 16;
  constexpr int NT = NB * (NB + 1) / 2;
  constexpr int NO = NB * (NB - 1) / 2;
  const int lane = threadIdx.x;
  int trow = 4 * (lane >> 4), tcol = lane & 15;
  if constexpr (kOpaqueStore<P, Q>) asm volatile("" : "+v"(trow), "+v"(tcol));
  const float fn = float(n);
  constexpr bool K3 = NB <= 3;
  // accR: Re (P1 in the three-product form); accI / accD: Im of the
  // off-diagonal / diagonal tiles (four-product form); p2, p3: P2 and P3
  f4 accR[NT], accI[(K3 || NO == 0) ? 1 : NO], accD[K3 ? 1 : NB];
  f4 p2[K3 ? NT : 1], p3[K3 ? NT : 1];
  // one chunk stream: the entering vectors' chunks, then the leaving ones';
  // chunk c + 1 is fetched while chunk c is accumulated.  Fetching one chunk
  // past the end reads the leaving list's kOut entries (KD > kMaxDelta + 6),
  // i.e. zeros, and is never used.
  const int na = (nadd + 3) >> 2, nch = na + ((nrem + 3) >> 2);
  __amdgpu_buffer_rsrc_t rs[NB];
#pragma unroll
  for (int I = 0; I < NB; ++I) rs[I] = block_rsrc<Q>(xwin, plane, rec, I);
  auto fetch = [&](int c, float2 (&v)[NB]) __attribute__((always_inline)) {
    const uint32_t off = (c < na ? sAdd + 4 * c : sRem + 4 * (c - na))[lane >> 4];
#pragma unroll
    for (int I = 0; I < NB; ++I) v[I] = bload(rs[I], loff[I] + off);
  };
  float2 vc[NB], vn[NB];
  fetch(0, vc);   // in flight while the old S is reloaded
  {
    int t = 0, u = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = I; J < NB; ++J) {
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int tr = trow + q4;
          float2 v = make_float2(0.f, 0.f);
          if (tile_in<P, Q>(I, J, tr, tcol)) v = tile_get<P, Q>(sS, I, J, tr, tcol);
          accR[t][q4] = v.x * fn;
          if constexpr (K3) {
            p2[t][q4] = 0.f;
            p3[t][q4] = (v.x + v.y) * fn;
          } else {
            if (J > I) accI[u][q4] = v.y * fn;
            else accD[I][q4] = v.y * fn;
          }
        }
        if (J > I) ++u;
        ++t;
      }
  }
#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    {
      fetch(ch + 1, vn);
      const float sg = ch < na ? 1.f : -1.f;
      float2 v[NB];
#pragma unroll
      for (int I = 0; I < NB; ++I) v[I] = vc[I];
#pragma unroll
      for (int I = 0; I < NB; ++I) vc[I] = vn[I];
      if constexpr (K3) {
        float xr[NB], xi[NB], a1[NB], a2[NB], a3[NB], b3[NB];
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          xr[I] = v[I].x;
          xi[I] = v[I].y;
          a1[I] = sg * v[I].x;
          a2[I] = sg * v[I].y;
          a3[I] = sg * (v[I].x + v[I].y);
          b3[I] = v[I].x - v[I].y;
        }
        int t = 0;
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = I; J < NB; ++J, ++t) {
            accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[I], xr[J], accR[t], 0, 0, 0);
            p2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[I], xi[J], p2[t], 0, 0, 0);
            p3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[I], b3[J], p3[t], 0, 0, 0);
          }
        continue;
      }
      float xr[NB], xi[NB], sxr[NB], sxi[NB], nsxr[NB];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        xr[I] = v[I].x;
        xi[I] = v[I].y;
        sxr[I] = sg * v[I].x;
        sxi[I] = sg * v[I].y;
        nsxr[I] = -sxr[I];
      }
      int t = 0, u = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = I; J < NB; ++J) {
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(sxr[I], xr[J], accR[t], 0, 0, 0);
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(sxi[I], xi[J], accR[t], 0, 0, 0);
          if (J > I) {
            accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(sxi[I], xr[J], accI[u], 0, 0, 0);
            accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(nsxr[I], xi[J], accI[u], 0, 0, 0);
            ++u;
          } else {
            accD[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(sxi[I], xr[I], accD[I], 0, 0, 0);
            accD[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(nsxr[I], xi[I], accD[I], 0, 0, 0);
          }
          ++t;
        }
    }
  }
  wave_sync();   // every lane has reloaded its part of the old S
  const float inv_n = 1.f / fn;
  {
    int t = 0, u = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = I; J < NB; ++J) {
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int tr = trow + q4;
          if (tile_keep<P, Q>(I, J, tr, tcol)) {
            float2 v;
            if constexpr (K3) {
              v.x = (accR[t][q4] + p2[t][q4]) * inv_n;
              v.y = (I == J && tr == tcol) ? 0.f : ((p3[t][q4] - accR[t][q4]) + p2[t][q4]) * inv_n;
            } else {
              v = make_float2(accR[t][q4] * inv_n, ((J > I) ? accI[u][q4] : accD[I][q4]) * inv_n);
            }
            tile_put<P, Q>(sS, I, J, tr, tcol, v);
            ssums_add<P, Q>(ss, I, J, I != J || tr != tcol, v);
          }
        }
        if (J > I) ++u;
        ++t;
      }
  }
  wave_sync();
}

// -------------------------------------------------------- a2, split BF16
// The same S from three BF16 products per tile: x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi); S ~ hi hi^H + hi lo^H + lo hi^H with FP32
// accumulation.  The split is done once per frame by split_planes into two
// planes in the layout of x, one packed BF16 pair (re, im) per complex
// sample: hi first, then lo.  The covariance kernel loads MFMA operands
// straight from them.  In a 16-vector chunk, 16-lane group g of the
// wavefront holds vectors 4g .. 4g + 3.
//   Re S tiles: v_mfma_f32_16x16x32_bf16 on Y = (re, im) pairs, which sums
//     re_I re_J + im_I im_J over the 16 vectors of the chunk.
//   Im S tiles: v_mfma_f32_16x16x16_bf16 on single components,
//     im_I re_J^T + (-re_I) im_J^T; the operands are half-word gathers (and
//     one sign flip) of the loaded pairs.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(const float2 (&v)[4], bf8& hi, bf8& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float a = v[e].x, b = v[e].y;
    const __bf16 ha = (__bf16)a, hb = (__bf16)b;
    hi[2 * e] = ha;
    hi[2 * e + 1] = hb;
    lo[2 * e] = (__bf16)(a - (float)ha);
    lo[2 * e + 1] = (__bf16)(b - (float)hb);
  }
}
__device__ __forceinline__ bf8 swap_neg(bf8 y) {
  u4 w = __builtin_bit_cast(u4, y);
#pragma unroll
  for (int e = 0; e < 4; ++e) w[e] = ((w[e] >> 16) | (w[e] << 16)) ^ 0x80000000u;
  return __builtin_bit_cast(bf8, w);
}

typedef short s4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));



// re (low halves) and im (high halves) of two packed pairs, as one dword
__device__ __forceinline__ uint32_t lo_halves(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x05040100u); }
__device__ __forceinline__ uint32_t hi_halves(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x07060302u); }

template <int P, int Q>
__device__ __forceinline__ void scm_bf16x3(const uint32_t* hwin, const uint32_t* lwin, int64_t plane, uint32_t rec,
                                           const uint32_t* sOffB, const uint32_t (&loff)[(P * Q + 15) / 16], int n,
                                           float2* sS, SSums<P>& ss) {
  constexpr int PQ = P * Q;
  constexpr int NB = (PQ + 15) / 16;
  constexpr int NT = NB * (NB + 1) / 2;
  const int lane = threadIdx.x;
  f4 accR[NT], accI[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) accR[t] = accI[t] = f4{0.f, 0.f, 0.f, 0.f};
  const int nch = (n + 15) >> 4;
  constexpr int PF = 2;
  u4 ring[PF][2][NB];   // hi / lo pairs of the lane's 4 vectors, per block
  __amdgpu_buffer_rsrc_t rh[NB], rl[NB];
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    const int64_t cb = int64_t((16 * I) / Q) * plane;
    rh[I] = __builtin_amdgcn_make_buffer_rsrc((void*)(hwin + cb), (short)0, int(rec), 0x00020000);
    rl[I] = __builtin_amdgcn_make_buffer_rsrc((void*)(lwin + cb), (short)0, int(rec), 0x00020000);
  }
  auto fetch = [&](int ch, u4 (&v)[2][NB]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t off = sOffB[ch * 16 + 4 * (lane >> 4) + e];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        v[0][I][e] = __builtin_amdgcn_raw_buffer_load_b32(rh[I], loff[I] + off, 0, 0);
        v[1][I][e] = __builtin_amdgcn_raw_buffer_load_b32(rl[I], loff[I] + off, 0, 0);
      }
    }
  };
  // MFMAs of one 16-vector chunk
  auto accumulate = [&](const u4 (&v)[2][NB]) {
    bf8 yh[NB], yl[NB];
    s4 reh[NB], rel[NB], imh[NB], iml[NB], nreh[NB], nrel[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      const u4 h = v[0][I], l = v[1][I];
      yh[I] = __builtin_bit_cast(bf8, h);
      yl[I] = __builtin_bit_cast(bf8, l);
      const u2 rh2{lo_halves(h[0], h[1]), lo_halves(h[2], h[3])};
      const u2 rl2{lo_halves(l[0], l[1]), lo_halves(l[2], l[3])};
      reh[I] = __builtin_bit_cast(s4, rh2);
      rel[I] = __builtin_bit_cast(s4, rl2);
      imh[I] = __builtin_bit_cast(s4, u2{hi_halves(h[0], h[1]), hi_halves(h[2], h[3])});
      iml[I] = __builtin_bit_cast(s4, u2{hi_halves(l[0], l[1]), hi_halves(l[2], l[3])});
      nreh[I] = __builtin_bit_cast(s4, u2{rh2[0] ^ 0x80008000u, rh2[1] ^ 0x80008000u});
      nrel[I] = __builtin_bit_cast(s4, u2{rl2[0] ^ 0x80008000u, rl2[1] ^ 0x80008000u});
    }
    int t = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = I; J < NB; ++J, ++t) {
        accR[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yh[I], yh[J], accR[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(imh[I], reh[J], accI[t], 0, 0, 0);
        accR[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yh[I], yl[J], accR[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nreh[I], imh[J], accI[t], 0, 0, 0);
        accR[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yl[I], yh[J], accR[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(imh[I], rel[J], accI[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(iml[I], reh[J], accI[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nreh[I], iml[J], accI[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nrel[I], imh[J], accI[t], 0, 0, 0);
      }
  };
#pragma unroll
  for (int s0 = 0; s0 < PF - 1; ++s0) {
    __builtin_amdgcn_sched_barrier(0);
    fetch(s0, ring[s0]);
  }
  int ch0 = 0;
  for (; ch0 + PF <= nch; ch0 += PF) {   // branch-free body, as in scm_fp32
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      __builtin_amdgcn_sched_barrier(0);
      fetch(ch0 + sl + PF - 1, ring[(sl + PF - 1) % PF]);
      __builtin_amdgcn_sched_barrier(0);   // all loads of the next chunk go out first
      accumulate(ring[sl]);
    }
  }
#pragma unroll
  for (int sl = 0; sl < PF - 1; ++sl)
    if (ch0 + sl < nch) accumulate(ring[sl]);
  const float inv_n = 1.f / float(n);
  // opaque, so that the element addresses are computed here for every pixel
  // rather than hoisted out of the caller's pixel loop and spilled
  int trow = 4 * (lane >> 4), tcol = lane & 15;
  asm volatile("" : "+v"(trow), "+v"(tcol));
  int t = 0;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = I; J < NB; ++J, ++t)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int tr = trow + q4;
        if (tile_keep<P, Q>(I, J, tr, tcol)) {
          const float2 v = make_float2(accR[t][q4] * inv_n, accI[t][q4] * inv_n);
          tile_put<P, Q>(sS, I, J, tr, tcol, v);
          ssums_add<P, Q>(ss, I, J, I != J || tr != tcol, v);
        }
      }
  wave_sync();
}

// ------------------------------------------------------------ kernel body
template <int Q>
struct Groups {
  static constexpr int QP = (Q <= 8) ? 8 : (Q <= 16) ? 16 : (Q <= 32) ? 32 : 64;
  static constexpr int G = 64 / QP;
};

template <bool B, typename T, typename F> struct Pick { using type = T; };
template <typename T, typename F> struct Pick<false, T, F> { using type = F; };

// True when the plan asks for more than the Kron-STAP statistic of one
// temporal steering (uniform across the grid).
__host__ __device__ __forceinline__ bool has_variants(const KParams& prm) {
  return prm.filter != 0 || prm.nbank != 0 || prm.passes != 1 || prm.E != nullptr || prm.bin != nullptr;
}

// Run mode: every output of a pixel outside the valid region is zero.
__device__ __forceinline__ void write_outside(const KParams& prm, int64_t idx) {
  prm.T[idx] = 0.f;
  if (prm.D) prm.D[idx] = 0;
  if (prm.E) prm.E[idx] = 0.f;
  if (prm.bin) prm.bin[idx] = 0;
  const int64_t hw = int64_t(prm.H) * prm.W;
  for (int k = 0; k < prm.passes; ++k) {
    if (prm.Tpass) prm.Tpass[k * hw + idx] = 0.f;
    if (prm.C && k > 0) prm.C[(k - 1) * hw + idx] = 0.f;
  }
}

// ------------------------------------------------ a6 + a8, batched
// Top-r_b time subspace, projected test vector and statistic for up to
// 64 / QP queued pixels of one wavefront: lane group `slot` (QP lanes) serves
// queue slot `slot`, whose lane k holds row k of the pixel's Hermitian time
// factor in Bq; slots >= nfill are empty.  Per slot the queue holds the pixel
// index, a flag (0 ok, 1 zero covariance, 2 non-finite), eta, the iteration
// count and U_A (p x RAM).  Writes T (and D, or the probe outputs).
// WAVE_LOCAL: other wavefronts of the workgroup run their own tails.
// vb: this lane's row of its slot's basis; on entry the warm start of the
// slots whose lanes set `keep` (the others start cold), on return the basis.
template <int P, int Q, int RBM, int MODE, typename EC, bool WAVE_LOCAL, bool VAR>
__device__ __forceinline__ void tail_batch(const KParams& prm, const float2 (&Bq)[Q], int slot, int nfill,
                                           const int* sQflag, const int64_t* sQidx, const float* sQeta,
                                           const int* sQit, const EC (*sQUA)[P * ((P < kMaxRA) ? P : kMaxRA)],
                                           EC* scratch, double tol, EC (&vb)[RBM], bool keep, bool& vb_ok) {
  using ES = decltype(EC{}.x);
  constexpr int RAM = (P < kMaxRA) ? P : kMaxRA;
  constexpr int QP = Groups<Q>::QP;
  const int tk = (threadIdx.x & 63) % QP;
  const int H = prm.H, W = prm.W;
  const int r_a = prm.r_a, r_b = prm.r_b;
  const bool slot_ok = slot < nfill;
  const bool rok = slot_ok && tk < Q;
  const int flag = slot_ok ? sQflag[slot] : 1;
  const int64_t pidx = slot_ok ? sQidx[slot] : 0;
  keep = keep && rok && flag == 0;
#pragma unroll
  for (int c = 0; c < RBM; ++c)
    if (!keep) vb[c] = czero<EC>();
  // FP64 solves iterate until converged where the r_b-th and next eigenvalues
  // of B lie close together (a ratio of 0.99 takes ~1 500 steps to 1e-10);
  // the loop exits on the step cap, so a group never runs unbounded
  constexpr int kTailSteps = sizeof(ES) == 8 ? 4000 : 200;
  if (r_b > 0)
    group_subspace<RBM, QP, Q, EC, WAVE_LOCAL>(Bq, rok && flag == 0, r_b, vb, scratch, true, kTailSteps, tol, keep);
  vb_ok = rok && flag == 0;
  // statistic
  int pr, pc;
  if (MODE == kModeRun) {
    pr = int(pidx / W);
    pc = int(pidx - int64_t(pr) * W);
  } else {
    pr = prm.pix[2 * pidx];
    pc = prm.pix[2 * pidx + 1];
  }
  const bool use = rok && flag == 0;
  // this lane's sample of every channel of the test snapshot
  const float2* xt = prm.x + (int64_t(pr) * W + pc) * Q;
  EC xv[P];
#pragma unroll
  for (int i = 0; i < P; ++i) xv[i] = use ? cto<EC>(xt[int64_t(i) * H * W * Q + tk]) : czero<EC>();
  const EC* Uq = sQUA[slot_ok ? slot : 0];   // U_A of the queued pixel, p x RAM
  // z <- (I - U_A U_A^H) z
  auto project_a = [&](EC (&z)[P]) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < RAM; ++c) {
      if (c >= r_a) continue;
      EC cw = czero<EC>();
#pragma unroll
      for (int i = 0; i < P; ++i) cw = ccfma(Uq[i * RAM + c], z[i], cw);
#pragma unroll
      for (int i = 0; i < P; ++i) z[i] = csub(z[i], cmul(Uq[i * RAM + c], cw));
    }
  };
  // fixed spatial steering: h and F_A h
  EC hs[P], fh[P];
  ES hfa = 0, hpa = 0;   // ||F_A h||^2, ||P_A h||^2
  if (prm.stat_mode != 0) {
#pragma unroll
    for (int i = 0; i < P; ++i) fh[i] = hs[i] = cto<EC>(prm.h_s[i]);
    project_a(fh);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      hfa += hs[i].x * fh[i].x + hs[i].y * fh[i].y;
      const EC ph = csub(hs[i], fh[i]);
      hpa += cabs2(ph);
    }
  }
  // Temporal steering: the plan's b_s, or each bin of a Doppler bank
  // b_m[k] = exp(2 pi j ((m k) mod M) / M); the statistic is the largest over
  // the bank, the bin its first maximiser.
  const int nbank = VAR ? prm.nbank : 0;
  const int nbins = nbank > 0 ? nbank : 1;
  const int K = VAR ? prm.passes : 1, PP = K > 1 ? P / K : P;
  const int filter = VAR ? prm.filter : 0;
  float* const Eout = VAR ? prm.E : nullptr;
  float T = 0.f, Ebest = 0.f;
  int best = 0;
  ES ez[P];   // per-channel energy |z_i|^2 / (b^H F_B b) at the best bin (passes > 1)
#pragma unroll
  for (int i = 0; i < P; ++i) ez[i] = 0;
  for (int m = 0; m < nbins; ++m) {
    EC bsk;
    ES bn2;
    if (nbank > 0) {
      const int ph = (m * tk) % nbank;
      float sn, cs;
      sincospif(float(2 * ph) / float(nbank), &sn, &cs);
      bsk = use ? cto<EC>(make_float2(cs, sn)) : czero<EC>();
      bn2 = ES(Q);
    } else {
      bsk = use ? cto<EC>(prm.b_s[tk]) : czero<EC>();
      bn2 = ES(prm.bs_norm2);
    }
    // g = F_B b
    EC gk = bsk;
    if (r_b > 0) {
#pragma unroll
      for (int c = 0; c < RBM; ++c) {
        if (c >= r_b) continue;
        const EC coef = gsum<QP>(ccfma(vb[c], bsk, czero<EC>()));
        if (use) gk = csub(gk, cmul(vb[c], coef));
      }
    }
    // w = X conj(g), z = F_A w
    EC w[P], z[P];
#pragma unroll
    for (int i = 0; i < P; ++i) z[i] = w[i] = gsum<QP>(cmul(xv[i], cconj(gk)));
    const ES den = gsum<QP>(ES(bsk.x * gk.x + bsk.y * gk.y));   // b^H F_B b
    project_a(z);
    const bool den_ok = den > ES(1e-12) * bn2;
    // w0 = X conj(b) (the classical filter, and channel 0's SAR image)
    EC w0[P];
    const int nw0 = filter == 1 ? P : (Eout ? 1 : 0);
#pragma unroll
    for (int i = 0; i < P; ++i) w0[i] = (i < nw0) ? gsum<QP>(cmul(xv[i], cconj(bsk))) : czero<EC>();
    ES t;
    if (filter == 0) {
      // Kron-STAP, Eq. (25): ||F_A X conj(F_B b)||^2 / (b^H F_B b)
      if (prm.stat_mode == 0) {
        ES num = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) num += cabs2(z[i]);
        t = den_ok ? num / den : ES(0);
      } else {
        EC hz = czero<EC>();
#pragma unroll
        for (int i = 0; i < P; ++i) hz = ccfma(hs[i], z[i], hz);
        const bool ok = den_ok && hfa > ES(1e-12) * ES(prm.h_norm2);
        t = ok ? cabs2(hz) / (hfa * den) : ES(0);
      }
    } else {
      // classical, Eq. (24): the GLRT over h reduces to
      // ||F_A X b*||^2 / ||b||^2 + ||P_A X conj(F_B b)||^2 / (b^H F_B b)
      EC z0[P];
#pragma unroll
      for (int i = 0; i < P; ++i) z0[i] = w0[i];
      project_a(z0);
      if (prm.stat_mode == 0) {
        ES n0 = 0, n1 = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          n0 += cabs2(z0[i]);
          n1 += cabs2(csub(w[i], z[i]));
        }
        t = n0 / bn2 + (den_ok ? n1 / den : ES(0));
      } else {
        // u = F_A X b* + P_A X conj(F_B b); h^H G h = ||F_A h||^2 ||b||^2 + ||P_A h||^2 b^H F_B b
        EC hu = czero<EC>();
#pragma unroll
        for (int i = 0; i < P; ++i) hu = ccfma(hs[i], cadd(z0[i], csub(w[i], z[i])), hu);
        const ES hgh = hfa * bn2 + hpa * (den_ok ? den : ES(0));
        t = hgh > ES(1e-12) * ES(prm.h_norm2) * bn2 ? cabs2(hu) / hgh : ES(0);
      }
    }
    if (m == 0 || float(t) > T) {
      T = float(t);
      best = m;
      if (Eout) {
        const ES isar = cabs2(w0[0]) / bn2;   // channel 0's matched-filter intensity
        Ebest = isar > ES(0) ? float(t / isar) : 0.f;
      }
      if (K > 1) {
#pragma unroll
        for (int i = 0; i < P; ++i) ez[i] = den_ok ? cabs2(z[i]) / den : ES(0);
      }
    }
  }
  if (!isfinite(T)) T = NAN;
  if (flag == 1) T = 0.f;
  if (flag == 2) T = NAN;
  if (slot_ok && tk == 0) {
    prm.T[pidx] = T;
    if (MODE == kModeRun) {
      if (prm.D) prm.D[pidx] = (T > prm.tau) ? 1 : 0;
      const int64_t hw = int64_t(H) * W;
      if (Eout) Eout[pidx] = flag == 2 ? NAN : (flag == 1 ? 0.f : Ebest);
      if (VAR && prm.bin) prm.bin[pidx] = uint8_t(flag == 0 ? best : 0);
      // pass k's image: the energy of its channels of z (passes > 1)
      if (K > 1 && (prm.Tpass || prm.C)) {
        ES t0 = 0;
#pragma unroll
        for (int i = 0; i < P; ++i)
          if (i < PP) t0 += ez[i];
#pragma unroll
        for (int k = 0; k < P; ++k) {
          if (k >= K) continue;
          ES ts = 0;
#pragma unroll
          for (int i = 0; i < P; ++i)
            if (i / PP == k) ts += ez[i];
          if (prm.Tpass) prm.Tpass[k * hw + pidx] = flag == 2 ? NAN : (flag == 1 ? 0.f : float(ts));
          if (prm.C && k > 0)
            prm.C[(k - 1) * hw + pidx] = flag == 2 ? NAN : (flag == 1 ? 0.f : float(sqrt(ts) - sqrt(t0)));
        }
      }
    }
    if (MODE == kModeProbe) {
      if (prm.eta) prm.eta[pidx] = sQeta[slot];
      if (prm.iters) prm.iters[pidx] = sQit[slot];
    }
  }
  if (MODE == kModeProbe && slot_ok) {
    if (prm.UA && tk < P) {
#pragma unroll
      for (int c = 0; c < RAM; ++c)
        if (c < r_a) prm.UA[(pidx * P + tk) * r_a + c] = (flag != 0) ? cz() : tof(sQUA[slot][tk * RAM + c]);
    }
    if (prm.UB && tk < Q) {
#pragma unroll
      for (int c = 0; c < RBM; ++c)
        if (c < r_b) prm.UB[(pidx * Q + tk) * r_b + c] = (flag != 0) ? cz() : tof(vb[c]);
    }
  }
  lds_sync<WAVE_LOCAL>();
}

// PREC 0: FP32 covariance, FP32 eigensolves and statistic.
// PREC 1: split-BF16 covariance, FP64 eigensolves and statistic.
// PREC 2: FP32 covariance (full sums, no sliding window), FP64 eigensolves
//         and statistic.
// LDS carve-out of one pixel pipeline (one workgroup), largest alignment first.
template <int P, int Q, int RBM, int PREC>
struct Lds {
  using EC = typename Pick<PREC != 0, double2, float2>::type;
  static constexpr int PQ = P * Q;
  static constexpr int RAM = (P < kMaxRA) ? P : kMaxRA;
  static constexpr int G = Groups<Q>::G;
  static constexpr int NB = (PQ + 15) / 16;
  // B / tail / transpose scratch: the raw time factor B (q x q), the batched
  // tail's basis exchange, and the FP32 path's diagonal-tile transpose
  static constexpr size_t kB = sizeof(float2) * Q * Q;
  static constexpr size_t kT = sizeof(EC) * RBM * Q * G;
  static constexpr size_t kP = PREC == 1 ? 0 : sizeof(float) * NB * 256;
  static constexpr size_t kBT = kB > kT ? (kB > kP ? kB : kP) : (kT > kP ? kT : kP);
  static constexpr size_t oUA = 0;                                        // EC[P*RAM]
  static constexpr size_t oAh = oUA + sizeof(EC) * P * RAM;               // EC[P*P]
  static constexpr size_t oQUA = oAh + sizeof(EC) * P * P;                // EC[G][P*RAM]
  static constexpr size_t oBT = oQUA + sizeof(EC) * G * P * RAM;          // kBT bytes
  static constexpr size_t oS = (oBT + kBT + 15) / 16 * 16;                // float2[P(P+1)/2][Q][Q+1]
  static constexpr size_t oA = oS + sizeof(float2) * (P * (P + 1) / 2) * Q * (Q + 1);   // float2[P*P]
  static constexpr size_t oQidx = oA + sizeof(float2) * P * P;            // int64[G]
  static constexpr size_t oOff = oQidx + sizeof(int64_t) * G;             // uint32[kMaxN + kOffPad]
  static constexpr size_t oDelta = oOff + sizeof(uint32_t) * (kMaxN + kOffPad);   // uint32[3][2][kMaxDelta + 8] (FP32)
  static constexpr size_t oQflag = oDelta + (PREC ? 0 : sizeof(uint32_t) * 6 * (kMaxDelta + 8));   // int[G]
  static constexpr size_t oQit = oQflag + sizeof(int) * G;                // int[G]
  static constexpr size_t oQeta = oQit + sizeof(int) * G;                 // float[G]
  static constexpr size_t bytes = ((oQeta + sizeof(float) * G) + 15) / 16 * 16;
};

// The whole per-pixel pass for `count` pixels starting at `first`: positions
// in the tiled order of the frame (run mode) or in the pixel list (probe
// mode).  One 64-lane workgroup; `lds` holds Lds<...>::bytes.
template <int P, int Q, int RBM, int MODE, int PREC, bool VAR = false>
__device__ __forceinline__ void run_pixels(const KParams& prm, int64_t first, int64_t count, char* lds) {
  using EC = typename Pick<PREC != 0, double2, float2>::type;   // eigensolver / statistic precision
  using ES = decltype(EC{}.x);
  using L = Lds<P, Q, RBM, PREC>;
  constexpr int PQ = P * Q;
  constexpr int NB = (PQ + 15) / 16;        // 16-row blocks of the pq x pq covariance
  constexpr int QQ = Q * Q;
  constexpr int NE = (QQ + 63) / 64;        // q x q entries per lane
  constexpr int RAM = L::RAM;
  constexpr int QP = Groups<Q>::QP;         // lanes per pixel in the batched tail
  constexpr int G = Groups<Q>::G;           // pixels per batched tail

  float2* const sS = reinterpret_cast<float2*>(lds + L::oS);     // S, upper blocks
  float2* const sBT = reinterpret_cast<float2*>(lds + L::oBT);   // raw B, then tail scratch
  uint32_t* const sOffB = reinterpret_cast<uint32_t*>(lds + L::oOff);
  // sliding window: per move, the entering then the leaving vectors
  uint32_t* const sDelta = reinterpret_cast<uint32_t*>(lds + L::oDelta);
  constexpr int KD = kMaxDelta + 8;
  float2* const sA = reinterpret_cast<float2*>(lds + L::oA);
  EC* const sUA = reinterpret_cast<EC*>(lds + L::oUA);
  EC* const sAh = reinterpret_cast<EC*>(lds + L::oAh);
  EC (*const sQUA)[P * RAM] = reinterpret_cast<EC (*)[P * RAM]>(lds + L::oQUA);   // queued pixels: U_A
  EC* const tail_scratch = reinterpret_cast<EC*>(sBT);
  int64_t* const sQidx = reinterpret_cast<int64_t*>(lds + L::oQidx);             //   pixel index
  int* const sQflag = reinterpret_cast<int*>(lds + L::oQflag);                   //   0 ok, 1 zero, 2 non-finite
  float* const sQeta = reinterpret_cast<float*>(lds + L::oQeta);
  int* const sQit = reinterpret_cast<int*>(lds + L::oQit);

  const int lane = threadIdx.x;
  const int n = prm.n;
  const int H = prm.H, W = prm.W;
  const int r_a = prm.r_a, r_b = prm.r_b;

  // byte offset of each stencil entry from the window origin (kOut past n);
  // samples are complex64 (8 bytes) or, on the mixed path, BF16 pairs (4)
  constexpr int kSample = PREC == 1 ? 4 : 8;
  wave_sync();
  for (int m = lane; m < kMaxN + kOffPad; m += 64)
    sOffB[m] = (m < n) ? uint32_t(((int(prm.st[2 * m]) * W + int(prm.st[2 * m + 1])) * Q - prm.st_min) * kSample)
                       : kOut;
  for (int m = lane; m < (PREC ? 0 : 6 * KD); m += 64) {
    const int t = m / KD, e = m - t * KD, mv = t >> 1;
    const int cnt = (t & 1) ? prm.nrem[mv] : prm.nadd[mv];
    uint32_t off = kOut;
    if (e < cnt) {   // cnt <= kMaxDelta
      const int dr = (t & 1) ? prm.drem[mv][2 * e] : prm.dadd[mv][2 * e];
      const int dc = (t & 1) ? prm.drem[mv][2 * e + 1] : prm.dadd[mv][2 * e + 1];
      off = uint32_t(((dr * W + dc) * Q - prm.st_min) * kSample);
    }
    sDelta[m] = off;
  }
  wave_sync();

  // Operand rows of this lane: row rho = 16*I + (lane & 15) of the stacked
  // snapshot, channel rho / q, sample rho % q; its byte offset inside block
  // I's record, which starts in channel 16*I / q.
  const int64_t plane = int64_t(H) * W * Q;
  uint32_t loff[NB];
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    const int rho = 16 * I + (lane & 15);
    const int ch = rho / Q, j = rho - ch * Q;
    loff[I] = (rho < PQ) ? uint32_t(((ch - (16 * I) / Q) * plane + j) * kSample) : kOut;
  }

  // queue of pixels waiting for the batched tail: lane (g, k) holds row k of
  // the Hermitian time factor of queued pixel g
  const int tg = lane / QP, tk = lane % QP;
  float2 Bq[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) Bq[l] = cz();
  int nq = 0;

  // ------------------------------------------------ a6 + a8 for G pixels
  // FP32 run mode: the queue holds the pixels of one sliding-window chain at
  // a time, and every batch of a chain but its first starts each slot from
  // the converged time-factor subspace of the previous batch's slot G-1-g,
  // its nearest pixel in the snake order of a unit (directly above it for
  // q = 16).  Like the sliding window, the choice depends only on the chain,
  // so the results are the same for every decomposition of the frame.
  constexpr bool kWarmTail = PREC == 0 && MODE == kModeRun;
  EC vbw[RBM];   // lane (g, k): row k of the basis that starts slot g
#pragma unroll
  for (int c = 0; c < RBM; ++c) vbw[c] = czero<EC>();
  bool vbw_ok = false;
  int64_t qchain = -1, bchain = -2;   // chain of the queued pixels, of the last batch
  auto tail = [&](int nfill) __attribute__((always_inline)) {
    const bool keep = kWarmTail && bchain == qchain && vbw_ok;
    bool ok;
    tail_batch<P, Q, RBM, MODE, EC, false, VAR>(prm, Bq, tg, nfill, sQflag, sQidx, sQeta, sQit, sQUA, tail_scratch,
                                                PREC ? 1e-10 : 2e-6, vbw, keep, ok);
    if constexpr (kWarmTail) {
      bchain = qchain;
      const int src = (G - 1 - tg) * QP + tk;
#pragma unroll
      for (int c = 0; c < RBM; ++c) {
        vbw[c].x = __shfl(vbw[c].x, src);
        vbw[c].y = __shfl(vbw[c].y, src);
      }
      vbw_ok = __shfl(int(ok), src) != 0;
    }
  };

  // Sliding window (run mode, FP32 path): every position of a chain but the
  // first is a one-pixel move from the one before it (tiled_move); such a
  // pixel updates the previous pixel's S when this workgroup has just
  // computed it from finite data.  A chain's first pixel takes the full sum,
  // and runs start on a chain, so the choice is the same for every
  // decomposition.
  bool chain = false;
  bool ua_ok = false;   // sUA holds the U_A of the pixel processed last
  for (int64_t it = 0; it < count; ++it) {
    int64_t idx;
    int r, c;
    const bool left_ok = chain;
    chain = false;
    if (MODE == kModeRun) {
      if (!tiled_pixel(first + it, H, W, &r, &c)) continue;
      idx = int64_t(r) * W + c;
    } else {
      idx = first + it;
      r = prm.pix[2 * idx];
      c = prm.pix[2 * idx + 1];
    }
    const bool valid = r >= prm.r0 && r < prm.r1 && c >= prm.c0 && c < prm.c1;
    if (!valid) {
      if (lane == 0) {
        if (MODE == kModeRun) write_outside(prm, idx);
        else prm.T[idx] = 0.f;
        if (MODE == kModeProbe) {
          if (prm.eta) prm.eta[idx] = 0.f;
          if (prm.iters) prm.iters[idx] = 0;
        }
      }
      if (MODE == kModeProbe) {
        if (prm.UA)
          for (int e = lane; e < P * r_a; e += 64) prm.UA[idx * P * r_a + e] = cz();
        if (prm.UB)
          for (int e = lane; e < Q * r_b; e += 64) prm.UB[idx * Q * r_b + e] = cz();
      }
      continue;
    }
    // window origin as a sample index (x and the split planes share the layout)
    const int64_t win = (int64_t(r) * W + c) * Q + prm.st_min;

    // ---------------------------------------------------------------- a2 SCM
    // (the FP64-solve paths are bound by their solves, not by the covariance
    // MFMAs, so they always take the full sum: no sliding-window residue)
    const int mv = tiled_move(first + it, H, W, kChainNarrow);
    const bool slide = PREC == 0 && MODE == kModeRun && left_ok && mv >= 0 && prm.nadd[0] >= 0;
    // q a multiple of 16: the block sums and ||S||^2 of a4 are gathered while
    // S is stored
    constexpr bool kSums = Q % 16 == 0;
    SSums<P> ss;
#pragma unroll
    for (int e = 0; e < P * P; ++e) ss.a0[e] = cz();
    ss.nr = 0.f;
    if constexpr (PREC != 1) {
      if (slide)
        scm_fp32_delta<P, Q>(prm.x + win, plane, prm.rec_bytes, sDelta + 2 * mv * KD, prm.nadd[mv],
                             sDelta + (2 * mv + 1) * KD, prm.nrem[mv], loff, n, sS, ss);
      else
        scm_fp32<P, Q>(prm.x + win, plane, prm.rec_bytes, sOffB, loff, n, sS, reinterpret_cast<float*>(sBT), ss);
    } else {
      scm_bf16x3<P, Q>(prm.xs + win, prm.xs + P * plane + win, plane, prm.rec_bytes / 2, sOffB, loff, n, sS, ss);
    }

    // ------------------------------------------------ a4 init, ||R||_F = ||S||_F
    float2 A[P * P];
    double normR2;
    {
      float2 a0[P * P];
      if constexpr (kSums) {
        normR2 = wsumd(double(ss.nr));
        // the upper block sums in one multi-value reduction
        constexpr int NU = P * (P + 1) / 2, NS = (2 * NU + 3) / 4 * 4;
        float sums[NS];
        {
          int e = 0;
#pragma unroll
          for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = i; j < P; ++j, e += 2) {
              sums[e] = ss.a0[i * P + j].x;
              sums[e + 1] = ss.a0[i * P + j].y;
            }
#pragma unroll
          for (int f = 2 * NU; f < NS; ++f) sums[f] = 0.f;
        }
        wsum_n<NS>(sums);
        {
          int e = 0;
#pragma unroll
          for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = i; j < P; ++j, e += 2) {
              a0[i * P + j] = cscale(make_float2(sums[e], sums[e + 1]), 1.f / float(QQ));
              if (j > i) a0[j * P + i] = cconj(a0[i * P + j]);
            }
        }
      } else {
#pragma unroll
        for (int e = 0; e < P * P; ++e) a0[e] = cz();
        float nr = 0.f;
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const int e = lane + 64 * t;
          if (e < QQ) {
            const int k = e / Q, l = e - (e / Q) * Q;
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
              for (int j = 0; j < P; ++j) {
                const float2 s = sget<P, Q>(sS, i, j, k, l);
                a0[i * P + j] = cadd(a0[i * P + j], s);
                nr += cabs2(s);
              }
          }
        }
        normR2 = wsumd(double(nr));
        constexpr int NS = (2 * P * P + 3) / 4 * 4;
        float sums[NS];
#pragma unroll
        for (int f = 0; f < NS; ++f) sums[f] = (f < 2 * P * P) ? ((f & 1) ? a0[f / 2].y : a0[f / 2].x) : 0.f;
        wsum_n<NS>(sums);
#pragma unroll
        for (int e = 0; e < P * P; ++e) a0[e] = cscale(make_float2(sums[2 * e], sums[2 * e + 1]), 1.f / float(QQ));
      }
      float an = 0.f;
#pragma unroll
      for (int e = 0; e < P * P; ++e) {
        A[e] = a0[e];
        an += cabs2(a0[e]);
      }
      if (double(an) <= 1e-24 * normR2) {   // fallback: partial trace R vec(I_q) (uniform branch)
        float2 pt[P * P];
#pragma unroll
        for (int e = 0; e < P * P; ++e) pt[e] = cz();
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const int e = lane + 64 * t;
          if (e < QQ && e / Q == e - (e / Q) * Q) {
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
              for (int j = 0; j < P; ++j) pt[i * P + j] = cadd(pt[i * P + j], sget<P, Q>(sS, i, j, e / Q, e / Q));
          }
        }
#pragma unroll
        for (int e = 0; e < P * P; ++e) A[e] = wsum(pt[e]);
      }
    }

    float eta = 0.f;
    int iters = 0;
    const bool zero = !(normR2 > 0.0);
    const bool bad = !isfinite(normR2);
    chain = !bad;   // this S may seed the next pixel's
    float2 bv[NE];
#pragma unroll
    for (int t = 0; t < NE; ++t) bv[t] = cz();

    if (!zero && !bad) {
      // --------------------------------------------------------- a5 LR-Kron
      float2 Ap[P * P];
      float bn2;
      double resid = 0.0;
      float anorm2 = 0.f;
#pragma unroll
      for (int e = 0; e < P * P; ++e) anorm2 += cabs2(A[e]);

      // one sweep over S: residual of (A, bv) if RES, then the new b and the
      // partial sums of R conj(b)
      auto sweep = [&](bool res) __attribute__((always_inline)) {
        const float ainv = xrcp(anorm2);
        float2 ap[P * P];
#pragma unroll
        for (int e = 0; e < P * P; ++e) ap[e] = cz();
        float bb = 0.f;
        double rr = 0.0;
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const int e = lane + 64 * t;
          if (QQ % 64 == 0 || e < QQ) {
            const int k = e / Q, l = e - (e / Q) * Q;
            float2 s[P * P];
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
              for (int j = 0; j < P; ++j) s[i * P + j] = sget<P, Q>(sS, i, j, k, l);
            if (res) {
              float acc = 0.f;
#pragma unroll
              for (int ij = 0; ij < P * P; ++ij) acc += cabs2(csub(s[ij], cmul(A[ij], bv[t])));
              rr += double(acc);
            }
            float2 bn = cz();
#pragma unroll
            for (int ij = 0; ij < P * P; ++ij) bn = ccfma(A[ij], s[ij], bn);
            bn = cscale(bn, ainv);
            bv[t] = bn;
            bb += cabs2(bn);
#pragma unroll
            for (int ij = 0; ij < P * P; ++ij) ap[ij] = ccfma(bn, s[ij], ap[ij]);
          } else {
            bv[t] = cz();
          }
        }
        // the 2 p^2 sums of R conj(b) and ||b||^2 in one multi-value reduction
        constexpr int NS = (2 * P * P + 1 + 3) / 4 * 4;
        float sums[NS];
#pragma unroll
        for (int ij = 0; ij < P * P; ++ij) {
          sums[2 * ij] = ap[ij].x;
          sums[2 * ij + 1] = ap[ij].y;
        }
#pragma unroll
        for (int e = 2 * P * P; e < NS; ++e) sums[e] = (e == 2 * P * P) ? bb : 0.f;
        wsum_n<NS>(sums);
        bn2 = sums[2 * P * P];
        const float binv = xrcp(bn2);
#pragma unroll
        for (int ij = 0; ij < P * P; ++ij) Ap[ij] = cscale(make_float2(sums[2 * ij], sums[2 * ij + 1]), binv);
        if (res) resid = wsumd(rr);
      };

      // EIG_{r_a}: A <- U (U^H A' U) U^H with U the top-r_a subspace of Herm(A').
      // A pixel that slides from its predecessor starts from that pixel's
      // U_A (sUA): the two training sets differ in a few vectors.  The choice
      // depends only on the chain position, as the sliding window does.
      const bool warm = slide && ua_ok;
      EC ua[P];
#pragma unroll
      for (int i = 0; i < P; ++i) ua[i] = warm ? sUA[i * RAM] : czero<EC>();
      auto eig_a = [&](bool cold) __attribute__((always_inline)) {
        EC Ah[P * P];
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
          for (int j = 0; j < P; ++j)
            Ah[i * P + j] = cscale(cadd(cto<EC>(Ap[i * P + j]), cconj(cto<EC>(Ap[j * P + i]))), ES(0.5));
        if (r_a == 1) {
          power_top<P, EC>([&](int i, int j) { return Ah[i * P + j]; }, ua, cold, 500, PREC ? 1e-12 : 2e-6);
          ES lam = 0;
#pragma unroll
          for (int i = 0; i < P; ++i) {
            EC s = czero<EC>();
#pragma unroll
            for (int j = 0; j < P; ++j) s = cfma(Ah[i * P + j], ua[j], s);
            lam += ua[i].x * s.x + ua[i].y * s.y;
          }
          anorm2 = 0.f;
#pragma unroll
          for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < P; ++j) {
              A[i * P + j] = tof(cscale(cmul(ua[i], cconj(ua[j])), lam));
              anorm2 += cabs2(A[i * P + j]);
            }
          // one lane writes U_A with static indices (a lane-indexed select
          // over ua[] is compiled into a scratch array)
          if (lane == 0) {
#pragma unroll
            for (int i = 0; i < P; ++i) sUA[i * RAM] = ua[i];
          }
          wave_sync();
          return;
        }
        // r_a > 1: the top-r_a subspace of Herm(A'), warm-started from the
        // previous U_A (in LDS).  p <= 4: every lane runs the same subspace
        // iteration with no cross-lane traffic; larger p: lane k holds row k
        // and the dot products are wave reductions (fewer registers).
        EC Vb[RAM][P];
        if (!cold) {
#pragma unroll
          for (int c = 0; c < RAM; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) Vb[c][i] = sUA[i * RAM + c];
        }
        wave_sync();
        if constexpr (P <= 4) {
          uniform_subspace<RAM, P, EC>([&](int i, int j) { return Ah[i * P + j]; }, r_a, Vb, cold, 500,
                                       PREC ? 1e-12 : 2e-6);
        } else {
          if (lane == 0) {
#pragma unroll
            for (int e = 0; e < P * P; ++e) sA[e] = tof(Ah[e]);
          }
          wave_sync();
          float2 mrow[P];
#pragma unroll
          for (int j = 0; j < P; ++j) mrow[j] = sA[(lane < P ? lane : 0) * P + j];
          // this lane's row of the warm start, read from LDS (a lane-indexed
          // select over Vb would be compiled into a scratch array)
          EC va[RAM];
#pragma unroll
          for (int c = 0; c < RAM; ++c) va[c] = (!cold && lane < P) ? sUA[lane * RAM + c] : czero<EC>();
          wave_sync();   // sUA is rewritten below
          group_subspace<RAM, 64, P, EC>(mrow, lane < P, r_a, va, sAh, cold, 500, PREC ? 1e-12 : 2e-6);
          // every lane gathers the whole basis from LDS
          if (lane < P) {
#pragma unroll
            for (int c = 0; c < RAM; ++c) sUA[lane * RAM + c] = va[c];
          }
          wave_sync();
#pragma unroll
          for (int c = 0; c < RAM; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) Vb[c][i] = sUA[i * RAM + c];
          wave_sync();
        }
        if (lane == 0) {
#pragma unroll
          for (int c = 0; c < RAM; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i)
              if (c < r_a) sUA[i * RAM + c] = Vb[c][i];
        }
        // Hs = U^H Herm(A') U and A = U Hs U^H
        EC Hs[RAM][RAM];
#pragma unroll
        for (int a = 0; a < RAM; ++a)
#pragma unroll
          for (int b = 0; b < RAM; ++b) {
            EC sacc = czero<EC>();
            if (a < r_a && b < r_a) {
#pragma unroll
              for (int i = 0; i < P; ++i) {
                EC t2 = czero<EC>();
#pragma unroll
                for (int j = 0; j < P; ++j) t2 = cfma(Ah[i * P + j], Vb[b][j], t2);
                sacc = ccfma(Vb[a][i], t2, sacc);
              }
            }
            Hs[a][b] = sacc;
          }
        anorm2 = 0.f;
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
          for (int j = 0; j < P; ++j) {
            EC sacc = czero<EC>();
#pragma unroll
            for (int a = 0; a < RAM; ++a) {
              if (a >= r_a) continue;
              EC t2 = czero<EC>();
#pragma unroll
              for (int b = 0; b < RAM; ++b)
                if (b < r_a) t2 = cfma(Hs[a][b], cconj(Vb[b][j]), t2);
              sacc = cfma(Vb[a][i], t2, sacc);
            }
            A[i * P + j] = tof(sacc);
            anorm2 += cabs2(A[i * P + j]);
          }
        wave_sync();
      };

      sweep(false);
      eig_a(!warm);
      iters = 1;
      double eta_prev = INFINITY;
      while (true) {
        sweep(true);
        const double e = sqrt(resid / normR2);
        eta = float(e);
        const bool stop = iters >= prm.max_iter ||
                          (prm.eps > 0.0 && iters >= prm.min_iter && fabs(e - eta_prev) <= prm.eps);
        if (stop) break;
        eta_prev = e;
        eig_a(false);
        ++iters;
      }
      // bv now holds the final b = R^T conj(a) / ||a||^2
    }
    ua_ok = !zero && !bad;

    // ------------------------------------------ enqueue for the batched tail
    // A full queue, or (warm tail) one that holds another chain's pixels,
    // runs its batch here, before this pixel joins: the queued pixels wait in
    // Bq and their own LDS slots, which this pixel's work does not touch, and
    // the tail is inlined at one place in the loop.
    wave_sync();   // S is dead from here on
    {
      bool flush = nq == G;
      int64_t cid = 0;
      if constexpr (kWarmTail) {
        cid = (first + it) / kChainNarrow;
        flush = flush || (nq > 0 && cid != qchain);
      }
      if (flush) {
        tail(nq);
        nq = 0;
      }
      if constexpr (kWarmTail) qchain = cid;
    }
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = lane + 64 * t;
      if (QQ % 64 == 0 || e < QQ) sBT[e] = bv[t];   // B[k][l] at k*q + l
    }
    wave_sync();
    if (tg == nq && tk < Q) {
#pragma unroll
      for (int l = 0; l < Q; ++l) Bq[l] = cscale(cadd(sBT[tk * Q + l], cconj(sBT[l * Q + tk])), 0.5f);
    }
    if (lane == 0) {
      sQidx[nq] = idx;
      sQflag[nq] = bad ? 2 : (zero ? 1 : 0);
      sQeta[nq] = eta;
      sQit[nq] = iters;
    }
    if (lane < P * RAM) sQUA[nq][lane] = (zero || bad) ? czero<EC>() : sUA[lane];
    wave_sync();
    ++nq;
  }
  if (nq > 0) tail(nq);
}

// Whole frame (run mode) or pixel list (probe mode).  Run mode: workgroup ids
// are remapped so each of the 8 XCDs takes a contiguous share of the frame.
// VAR: the statistic variants (filter, Doppler bank, enhancement, passes) are
// compiled into a kernel of their own, so that the plain statistic keeps its
// register budget.
template <int P, int Q, int RBM, int MODE, int PREC, bool VAR = false>
__global__ __launch_bounds__(64, 2) void kstap_kernel(const KParams prm) {
  __shared__ __attribute__((aligned(16))) char lds[Lds<P, Q, RBM, PREC>::bytes];
  int64_t first, count;
  if (MODE == kModeRun) {
    const int per = gridDim.x >> 3;   // grid is a multiple of 8 (one share per XCD)
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (logical >= prm.nlogical) return;
    const int64_t total = tiled_positions(prm.H, prm.W);
    first = int64_t(logical) * prm.pix_per_block;
    count = total - first;
    if (count > prm.pix_per_block) count = prm.pix_per_block;
  } else {
    first = int64_t(blockIdx.x) * prm.pix_per_block;
    count = prm.npix - first;
    if (count > prm.pix_per_block) count = prm.pix_per_block;
  }
  run_pixels<P, Q, RBM, MODE, PREC, VAR>(prm, first, count, lds);
}

// Persistent batched kernel: every workgroup pops work items (runs of `ppb`
// consecutive tiled-order positions of one tile's range [range_first,
// range_end)) from a
// device counters until every queue is empty (kQueues queues, see kstap_internal.h).  Items are numbered tile after
// tile in the order of `order` (longest tiles first); prefix[j] is the first item of order[j] (prefix[nt] = total).
template <int P, int Q, int RBM, int PREC>
__global__ __launch_bounds__(64, 2) void kstap_persistent(const KParams* __restrict__ descs,
                                                          const int32_t* __restrict__ order,
                                                          const int64_t* __restrict__ prefix, int nt,
                                                          int ppb, unsigned long long* counter) {
  __shared__ __attribute__((aligned(16))) char lds[Lds<P, Q, RBM, PREC>::bytes];
  __shared__ long long s_item;
  const int64_t total = prefix[nt];
  // queue q holds items [total q / kQueues, total (q + 1) / kQueues); start
  // with this workgroup's XCD (dispatch is round-robin over the XCDs), then
  // move on whenever a queue is empty: every workgroup leaves after finding
  // all kQueues queues empty
  int q = int(blockIdx.x % kQueues), empty = 0;
  while (true) {
    const int64_t qlo = total * q / kQueues, qhi = total * (q + 1) / kQueues;
    if (threadIdx.x == 0) s_item = (long long)atomicAdd(counter + q, 1ull);
    wave_sync();
    const int64_t item = qlo + s_item;
    wave_sync();
    if (item >= qhi) {
      if (++empty == kQueues) break;
      q = (q + 1) % kQueues;
      continue;
    }
    int lo = 0, hi = nt - 1;   // last j with prefix[j] <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const KParams& prm = descs[order[lo]];
    const int64_t first = prm.range_first + (item - prefix[lo]) * ppb;
    int64_t count = prm.range_end - first;
    if (count > ppb) count = ppb;
    run_pixels<P, Q, RBM, kModeRun, PREC>(prm, first, count, lds);
  }
}

// ====================================================================
// Wide pixels (p*q > 64): one 512-lane workgroup (8 wavefronts) per pixel.
//
// The covariance tiles (16 x 16, upper block-triangle) are dealt round-robin
// to the 8 waves.  Training vectors are staged in LDS 16 at a time (split
// BF16 hi/lo pairs for PREC 1, FP32 for PREC 0), double-buffered: the global
// loads of the next chunk are in flight while the waves run the MFMAs of the
// current one.  S is kept as its upper q x q blocks S(i,j), i <= j (the lower
// blocks are their conjugate transposes), which halves its LDS footprint, and
// it outlives the pixel: in run mode every pixel of a sliding-window chain
// but the first starts from the previous pixel's n*S (a one-pixel move) and
// stages only the training vectors that enter the stencil (added) and leave
// it (subtracted), as the narrow FP32 kernels do.  LR-Kron sweeps run over all 512 lanes with the
// block sums reduced across waves through LDS; the small factor-A solves are
// computed identically by every wave.  The Hermitian time factors are queued
// in LDS and the batched tail (a6 + a8) runs 64/q' pixels per wave on waves
// 0-3 at once.  Eight waves (two per SIMD, the LDS footprint allows one
// workgroup per compute unit) hide each other's LDS, reduction and barrier
// latencies; with four, each SIMD ran a single wave.
// ====================================================================
constexpr int kWideWaves = 8;                      // waves per wide workgroup
constexpr int kWideThreads = 64 * kWideWaves;
constexpr int kTailWaves = 4;                      // waves that run the batched tail

template <int P, int Q, int RBM, int PREC>
struct WideLds {
  using EC = typename Pick<PREC == 1, double2, float2>::type;
  static constexpr int PQ = P * Q;
  static constexpr int NB = (PQ + 15) / 16;
  static constexpr int NBLK = P * (P + 1) / 2;
  static constexpr int RAM = (P < kMaxRA) ? P : kMaxRA;
  static constexpr int G = Groups<Q>::G;
  static constexpr int NQ = kTailWaves * G;                          // pixels per batched tail
  static constexpr size_t kS = sizeof(float2) * NBLK * Q * (Q + 1);  // upper blocks of S
  static constexpr size_t rowb = PREC ? 80 : 144;                    // padded bytes per staged row
  static constexpr size_t stage1 = PREC ? 2 * NB * 16 * rowb : NB * 16 * rowb;   // hi + lo, or fp32
  static constexpr size_t kStage = 2 * stage1;
  static constexpr size_t kTail = sizeof(EC) * RBM * Q * G * kTailWaves;   // subspace scratch of the tail waves
  static constexpr size_t kST = kStage > kTail ? kStage : kTail;
  static constexpr size_t oS = 0;
  static constexpr size_t oStage = (kS + 15) / 16 * 16;              // staging; tail scratch between pixels
  static constexpr size_t oHq = oStage + (kST + 15) / 16 * 16;       // float2[NQ][Q*Q]: queued Herm(B)
  static constexpr size_t oQUA = oHq + sizeof(float2) * NQ * Q * Q;  // EC[NQ][P*RAM]: queued U_A
  static constexpr size_t oUA = oQUA + sizeof(EC) * NQ * P * RAM;    // EC[P*RAM]
  static constexpr size_t oAh = oUA + sizeof(EC) * P * RAM;          // EC[P*P]
  static constexpr size_t oRedD = oAh + sizeof(EC) * P * P;          // double[kWideWaves]
  static constexpr size_t oQidx = oRedD + sizeof(double) * kWideWaves;   // int64[NQ]
  static constexpr size_t oRed = oQidx + sizeof(int64_t) * NQ;       // float[kWideWaves][KRED]
  static constexpr int KRED = 2 * P * P + 8;
  static constexpr size_t oA = oRed + sizeof(float) * kWideWaves * KRED;   // float2[P*P]
  static constexpr size_t oAp = oA + sizeof(float2) * P * P;         // float2[P*P]: block sums (A_0, R b*)
  static constexpr size_t oB = oAp + sizeof(float2) * P * P;         // float2[Q*Q]: current b
  static constexpr size_t oOff = oB + sizeof(float2) * Q * Q;        // int[kMaxN]
  static constexpr size_t oDel = oOff + sizeof(int) * kMaxN;         // int[3][2*kMaxDelta]: per move, entering, leaving
  static constexpr size_t oQflag = oDel + sizeof(int) * 6 * kMaxDelta;   // int[NQ]
  static constexpr size_t oQit = oQflag + sizeof(int) * NQ;          // int[NQ]
  static constexpr size_t oQeta = oQit + sizeof(int) * NQ;           // float[NQ]
  static constexpr size_t bytes = (oQeta + sizeof(float) * NQ + 15) / 16 * 16;
  static_assert(bytes <= 160 * 1024, "LDS of one workgroup");
};

__device__ __forceinline__ void block_sync() { __syncthreads(); }

// Sums a double over the lanes of the workgroup (every lane gets the sum).
__device__ __forceinline__ double block_sumd(double v, double* red) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  v = wsumd(v);
  if (lane == 0) red[w] = v;
  block_sync();
  v = 0.0;
#pragma unroll
  for (int i = 0; i < kWideWaves; ++i) v += red[i];
  block_sync();
  return v;
}

template <int P, int Q, int RBM, int MODE, int PREC, bool VAR = false>
__device__ __forceinline__ void run_pixels_wide(const KParams& prm, int64_t first, int64_t count, char* lds) {
  using EC = typename Pick<PREC == 1, double2, float2>::type;
  using ES = decltype(EC{}.x);
  using L = WideLds<P, Q, RBM, PREC>;
  constexpr int PQ = P * Q;
  constexpr int NB = L::NB;
  constexpr int QS = Q + 1;
  constexpr int QQ = Q * Q;
  constexpr int NE = (QQ + kWideThreads - 1) / kWideThreads;   // q x q entries per lane
  constexpr int RAM = L::RAM;
  constexpr int NPAIR = NB * (NB + 1) / 2;
  constexpr int MYP = (NPAIR + kWideWaves - 1) / kWideWaves;   // tile pairs per wave (round-robin)
  constexpr int QP = Groups<Q>::QP;
  constexpr int G = L::G;
  constexpr int NQ = L::NQ;

  float2* const sS = reinterpret_cast<float2*>(lds + L::oS);
  char* const stage = lds + L::oStage;
  float* const red = reinterpret_cast<float*>(lds + L::oRed);
  double* const redd = reinterpret_cast<double*>(lds + L::oRedD);
  EC* const sUA = reinterpret_cast<EC*>(lds + L::oUA);
  EC* const sAh = reinterpret_cast<EC*>(lds + L::oAh);
  float2* const sA = reinterpret_cast<float2*>(lds + L::oA);
  float2* const sAp = reinterpret_cast<float2*>(lds + L::oAp);
  float2* const sB = reinterpret_cast<float2*>(lds + L::oB);
  int* const sOff = reinterpret_cast<int*>(lds + L::oOff);
  int* const sDel = reinterpret_cast<int*>(lds + L::oDel);
  float2* const sHq = reinterpret_cast<float2*>(lds + L::oHq);
  EC (*const sQUA)[P * RAM] = reinterpret_cast<EC (*)[P * RAM]>(lds + L::oQUA);
  int64_t* const sQidx = reinterpret_cast<int64_t*>(lds + L::oQidx);
  int* const sQflag = reinterpret_cast<int*>(lds + L::oQflag);
  int* const sQit = reinterpret_cast<int*>(lds + L::oQit);
  float* const sQeta = reinterpret_cast<float*>(lds + L::oQeta);

  // the wave index is uniform: keep it (and the tile pairs below) in SGPRs
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  constexpr int NL = (QQ + 63) / 64;   // q x q block entries per lane in the block passes
  const int n = prm.n, H = prm.H, W = prm.W;
  const int r_a = prm.r_a, r_b = prm.r_b;

  // sample offsets of the stencil, and per one-pixel move those of the
  // entering then the leaving vectors
  block_sync();
  for (int m = tid; m < n; m += kWideThreads) sOff[m] = (int(prm.st[2 * m]) * W + int(prm.st[2 * m + 1])) * Q;
  for (int m = tid; m < 6 * kMaxDelta; m += kWideThreads) {
    const int mv = m / (2 * kMaxDelta), e = m - mv * (2 * kMaxDelta);
    int off = 0;
    if (prm.nadd[0] >= 0) {
      const int na = prm.nadd[mv], nr = prm.nrem[mv];   // each <= kMaxDelta
      if (e < na) off = (int(prm.dadd[mv][2 * e]) * W + int(prm.dadd[mv][2 * e + 1])) * Q;
      else if (e < na + nr) off = (int(prm.drem[mv][2 * (e - na)]) * W + int(prm.drem[mv][2 * (e - na) + 1])) * Q;
    }
    sDel[m] = off;
  }
  block_sync();

  // this wave's tile pairs (I, J), I <= J, round-robin over the upper tiles
  int pI[MYP], pJ[MYP];
  bool pOk[MYP];
  {
    int t = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = I; J < NB; ++J, ++t) {
        if (t % kWideWaves == wave) {
          pI[t / kWideWaves] = I;
          pJ[t / kWideWaves] = J;
        }
      }
#pragma unroll
    for (int u = 0; u < MYP; ++u) pOk[u] = (u * kWideWaves + wave) < NPAIR;
  }

  constexpr int NIT = (16 * PQ + kWideThreads - 1) / kWideThreads;
  const int64_t plane = int64_t(H) * W * Q;

  // ------------------------------------------ a6 + a8 for the queued pixels
  // wave w < kTailWaves serves queue slots w*G .. w*G + G - 1; lane k of a
  // slot's group takes row k of its Hermitian time factor (column k,
  // conjugated: the stored factor is exactly Hermitian)
  auto tail = [&](int nfill) __attribute__((always_inline)) {
    int lanev = threadIdx.x & 63;
    asm volatile("" : "+v"(lanev));   // per call: no lane arithmetic hoisted out of the pixel loop
    const int lane = lanev;
    if (wave < kTailWaves) {   // uniform per wave; the tail syncs inside a wave only
      const int slot = wave * G + lane / QP, tk = lane % QP;
      const bool own = slot < nfill && tk < Q;
      float2 Bq[Q];
#pragma unroll
      for (int l = 0; l < Q; ++l) Bq[l] = own ? cconj(sHq[(slot < nfill ? slot : 0) * QQ + l * Q + tk]) : cz();
      EC* const scr = reinterpret_cast<EC*>(stage) + wave * (RBM * Q * G);
      EC vb[RBM];
      bool vb_ok;
      tail_batch<P, Q, RBM, MODE, EC, true, VAR>(prm, Bq, slot, nfill, sQflag, sQidx, sQeta, sQit, sQUA, scr,
                                                 PREC ? 1e-10 : 2e-6, vb, false, vb_ok);
    }
    block_sync();
  };

  int nq = 0;
  bool chain = false;   // the previous position left a usable S in LDS
  bool ua_ok = false;   // sUA holds the U_A of the pixel processed last
  auto pixel = [&](int64_t itp) __attribute__((always_inline)) {
    // Opaque per-pixel copy of the thread index: the index arithmetic below
    // (staging items, tile elements, q x q entries) is redone for every pixel
    // rather than hoisted out of the pixel loop, where at two waves per SIMD
    // it would not fit in registers.
    int tidv = threadIdx.x;
    asm volatile("" : "+v"(tidv));
    const int tid = tidv, lane = tidv & 63;
    // staging items of this thread: (vector v, row rho) = divmod(tid + 512 it, PQ)
    auto item = [&](int it, int* v, int* rho) __attribute__((always_inline)) -> bool {
      const int e = tid + kWideThreads * it;
      *v = e / PQ;
      *rho = e - *v * PQ;
      return e < 16 * PQ;
    };
    int64_t idx;
    int r, c;
    const bool left_ok = chain;
    chain = false;
    if (MODE == kModeRun) {
      if (!tiled_pixel(first + itp, H, W, &r, &c)) return;
      idx = int64_t(r) * W + c;
    } else {
      idx = first + itp;
      r = prm.pix[2 * idx];
      c = prm.pix[2 * idx + 1];
    }
    const bool valid = r >= prm.r0 && r < prm.r1 && c >= prm.c0 && c < prm.c1;
    if (!valid) {
      if (tid == 0) {
        if (MODE == kModeRun) write_outside(prm, idx);
        else prm.T[idx] = 0.f;
        if (MODE == kModeProbe) {
          if (prm.eta) prm.eta[idx] = 0.f;
          if (prm.iters) prm.iters[idx] = 0;
        }
      }
      if (MODE == kModeProbe) {
        if (prm.UA)
          for (int e = tid; e < P * r_a; e += kWideThreads) prm.UA[idx * P * r_a + e] = cz();
        if (prm.UB)
          for (int e = tid; e < Q * r_b; e += kWideThreads) prm.UB[idx * Q * r_b + e] = cz();
      }
      return;
    }
    const float2* xp = prm.x + (int64_t(r) * W + c) * Q;

    // ------------------------------------------------------------ a2 SCM
    // Full sum over the n stencil vectors, or (sliding window, a one-pixel
    // move inside a unit) the previous pixel's n*S plus the entering vectors
    // minus the leaving ones: list entries m < npos are added, the others
    // subtracted.
    const int mv = tiled_move(first + itp, H, W, kChainWide);
    const bool slide = MODE == kModeRun && left_ok && mv >= 0 && prm.nadd[0] >= 0;
    const int* const list = slide ? sDel + mv * 2 * kMaxDelta : sOff;
    // EIG_{r_a} of a pixel that slides from its predecessor starts from that
    // pixel's U_A (sUA); the choice follows the chain, as the sliding window
    const bool warm = slide && ua_ok;
    const int cnt = slide ? prm.nadd[mv] + prm.nrem[mv] : n;
    const int npos = slide ? prm.nadd[mv] : n;
    const float fn = float(n);
    // this lane's row and column inside a 16 x 16 tile.  On the mixed path
    // they are made opaque, so that the S element addresses below are computed
    // here, per pixel, instead of being hoisted out of the pixel loop (72 more
    // live registers there, which spilled); the FP32 path has room for them.
    int trow = 4 * (lane >> 4), tcol = lane & 15;
    if constexpr (PREC == 1) asm volatile("" : "+v"(trow), "+v"(tcol));
    f4 accR[MYP], accI[MYP];
#pragma unroll
    for (int u = 0; u < MYP; ++u) {
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        // element (a, b) of the old S, read from its upper block (conjugated
        // when it lies below the block diagonal), without branches
        const int a = 16 * pI[u] + trow + q4, b = 16 * pJ[u] + tcol;
        const int ba = a / Q, bb = b / Q, ka = a - ba * Q, kb = b - bb * Q;
        const bool upper = ba <= bb;
        const int off = upper ? sblk<P, Q>(ba, bb) + ka * QS + kb : sblk<P, Q>(bb, ba) + kb * QS + ka;
        const bool use = slide && pOk[u] && a < PQ && b < PQ;
        const float2 v = sS[use ? off : 0];
        accR[u][q4] = use ? v.x * fn : 0.f;
        accI[u][q4] = use ? (upper ? v.y : -v.y) * fn : 0.f;
      }
    }
    const int nch = (cnt + 15) >> 4;
    float2 pre[NIT];
    auto gload = [&](int ch) __attribute__((always_inline)) {
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int v, rho;
        const bool in = item(it, &v, &rho);
        const int m = ch * 16 + v;
        const bool ok = in && m < cnt;
        const int chn = rho / Q;
        pre[it] = load_or_zero(xp + chn * plane + (rho - chn * Q) + list[ok ? m : 0], ok);
      }
    };
    auto sstore = [&](int buf) __attribute__((always_inline)) {
      char* base = stage + buf * L::stage1;
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int v, rho;
        if (!item(it, &v, &rho)) continue;
        if constexpr (PREC == 1) {
          const float a = pre[it].x, b = pre[it].y;
          const __bf16 ha = (__bf16)a, hb = (__bf16)b;
          const __bf16 la = (__bf16)(a - (float)ha), lb = (__bf16)(b - (float)hb);
          __bf16* hrow = reinterpret_cast<__bf16*>(base + size_t(rho) * L::rowb);
          __bf16* lrow = reinterpret_cast<__bf16*>(base + size_t(NB * 16 + rho) * L::rowb);
          hrow[2 * v] = ha;
          hrow[2 * v + 1] = hb;
          lrow[2 * v] = la;
          lrow[2 * v + 1] = lb;
        } else {
          float2* row = reinterpret_cast<float2*>(base + size_t(rho) * L::rowb);
          row[v] = pre[it];
        }
      }
    };
    gload(0);
    sstore(0);
    block_sync();
    for (int ch = 0; ch < nch; ++ch) {
      const int buf = ch & 1;
      if (ch + 1 < nch) gload(ch + 1);
      const char* base = stage + buf * L::stage1;
      const int g = lane >> 4, rr = lane & 15;
      if constexpr (PREC == 1) {
        // operand of block I: row 16 I + rr, vectors 4g..4g+3 (re, im) = 16 bytes;
        // the row operand of a subtracted vector is negated (sign bits of its pair)
        u4 msk;
#pragma unroll
        for (int e = 0; e < 4; ++e) msk[e] = (ch * 16 + 4 * g + e >= npos) ? 0x80008000u : 0u;
        auto ld = [&](int I, bool lo) __attribute__((always_inline)) -> u4 {
          const int row = 16 * I + rr;
          if (row >= PQ) return u4{0u, 0u, 0u, 0u};
          const char* p = base + size_t((lo ? NB * 16 : 0) + row) * L::rowb + g * 16;
          return *reinterpret_cast<const u4*>(p);
        };
#pragma unroll
        for (int u = 0; u < MYP; ++u) {
          if (!pOk[u]) continue;
          const bf8 hI = __builtin_bit_cast(bf8, ld(pI[u], false) ^ msk);
          const bf8 lI = __builtin_bit_cast(bf8, ld(pI[u], true) ^ msk);
          const bf8 hJ = __builtin_bit_cast(bf8, ld(pJ[u], false)), lJ = __builtin_bit_cast(bf8, ld(pJ[u], true));
          const bf8 zh = swap_neg(hI), zl = swap_neg(lI);
          accR[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hI, hJ, accR[u], 0, 0, 0);
          accI[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh, hJ, accI[u], 0, 0, 0);
          accR[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hI, lJ, accR[u], 0, 0, 0);
          accI[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zh, lJ, accI[u], 0, 0, 0);
          accR[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lI, hJ, accR[u], 0, 0, 0);
          accI[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zl, hJ, accI[u], 0, 0, 0);
        }
      } else {
        // 4 K-steps of 4 vectors: lane (row rr, vector 4 s + g)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const float sg = (ch * 16 + 4 * s4 + g >= npos) ? -1.f : 1.f;
          auto ld = [&](int I) __attribute__((always_inline)) -> float2 {
            const int row = 16 * I + rr;
            if (row >= PQ) return cz();
            return reinterpret_cast<const float2*>(base + size_t(row) * L::rowb)[4 * s4 + g];
          };
#pragma unroll
          for (int u = 0; u < MYP; ++u) {
            if (!pOk[u]) continue;
            const float2 a = cscale(ld(pI[u]), sg), b = ld(pJ[u]);
            accR[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, accR[u], 0, 0, 0);
            accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, accI[u], 0, 0, 0);
            accR[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, accR[u], 0, 0, 0);
            accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.x, b.y, accI[u], 0, 0, 0);
          }
        }
      }
      if (ch + 1 < nch) sstore(buf ^ 1);
      block_sync();
    }
    // S to LDS as upper blocks: every element (a, b), a <= b, has one writer
    // (the staging barrier above also ends every wave's reload of the old S)
    block_sync();
    {
      if constexpr (PREC == 1) asm volatile("" : "+v"(trow), "+v"(tcol));   // as above
      const float inv_n = 1.f / fn;
#pragma unroll
      for (int u = 0; u < MYP; ++u) {
        if (!pOk[u]) continue;
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int a = 16 * pI[u] + trow + q4, b = 16 * pJ[u] + tcol;
          if (a < PQ && b < PQ && a <= b) sput<P, Q>(sS, a, b, make_float2(accR[u][q4] * inv_n, accI[u][q4] * inv_n));
        }
      }
    }
    block_sync();

    // S(i,j)[k][l] for any (i, j)
    auto Sget = [&](int i, int j, int k, int l) __attribute__((always_inline)) -> float2 {
      if (i <= j) return sS[((i * P - i * (i - 1) / 2 + (j - i)) * Q + k) * QS + l];
      return cconj(sS[((j * P - j * (j - 1) / 2 + (i - j)) * Q + l) * QS + k]);
    };

    // Block pass: out[ij] = scale * sum_kl conj(w_kl) S(i,j)_kl for the P*P
    // blocks, dealt round-robin to the waves; a wave's lanes split the q x q
    // entries (this lane: e = lane + 64 m, weight wv[m]) and reduce with DPP.
    // Optionally accumulates sum |S(i,j)_kl|^2 of the visited entries in *nr.
    // out[] is complete after the next block_sync.
    // The wave's blocks are accumulated first and reduced together, so the
    // DPP reduction chains of different blocks overlap.
    auto block_pass = [&](const float2 (&wv)[NL], float scale, float2* out, double* nr) {
      constexpr int NU = (P * P + kWideWaves - 1) / kWideWaves;
      float2 acc[NU];
      double n2 = 0.0;   // exact squares of the FP32 entries, FP64 sums
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        acc[u] = cz();
        const int ij = wave + kWideWaves * u;
        if (ij < P * P) {   // uniform per wave
          const int i = ij / P, j = ij - (ij / P) * P;
          const bool up = i <= j;
          const int a = up ? i : j, b = up ? j : i;
          const int base = (a * P - a * (a - 1) / 2 + (b - a)) * Q * QS;
#pragma unroll
          for (int m = 0; m < NL; ++m) {
            if (lane + 64 * m < QQ) {
              const int e = lane + 64 * m;
              int k = e / Q, l = e - (e / Q) * Q;
              asm volatile("" : "+v"(k), "+v"(l));
              float2 sv = sS[base + (up ? k * QS + l : l * QS + k)];
              sv.y = up ? sv.y : -sv.y;
              acc[u] = ccfma(wv[m], sv, acc[u]);
              if (nr) n2 = fma(double(sv.x), double(sv.x), fma(double(sv.y), double(sv.y), n2));
            }
          }
        }
      }
      if (nr) *nr += n2;
      {
        constexpr int NS = (2 * NU + 3) / 4 * 4;
        float sums[NS];
#pragma unroll
        for (int f = 0; f < NS; ++f) sums[f] = (f < 2 * NU) ? ((f & 1) ? acc[f / 2].y : acc[f / 2].x) : 0.f;
        wsum_n<NS>(sums);
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[u] = make_float2(sums[2 * u], sums[2 * u + 1]);
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int ij = wave + kWideWaves * u;
        if (ij < P * P && lane == 0) out[ij] = cscale(acc[u], scale);
      }
    };

    // ------------------------------------------------ a4 init, ||R||_F = ||S||_F
    // The current space factor A lives in LDS (sA, P x P): every lane reads
    // it, as broadcasts, in the sweeps.
    double normR2;
    {
      float2 wv[NL];
#pragma unroll
      for (int m = 0; m < NL; ++m) wv[m] = make_float2(1.f, 0.f);
      double nr = 0.0;
      block_pass(wv, 1.f / float(QQ), sAp, &nr);
      normR2 = block_sumd(nr, redd);   // its barriers also publish sAp
      float an = 0.f;
#pragma unroll
      for (int e = 0; e < P * P; ++e) an += cabs2(sAp[e]);
      if (double(an) <= 1e-24 * normR2) {   // fallback: partial trace R vec(I_q)
#pragma unroll
        for (int m = 0; m < NL; ++m) {
          const int e = lane + 64 * m;
          wv[m] = (e < QQ && e / Q == e - (e / Q) * Q) ? make_float2(1.f, 0.f) : cz();
        }
        block_sync();
        block_pass(wv, 1.f, sAp, nullptr);
        block_sync();
      }
      if (tid < P * P) sA[tid] = sAp[tid];
      block_sync();
    }

    float eta = 0.f;
    int iters = 0;
    const bool zero = !(normR2 > 0.0);
    const bool bad = !isfinite(normR2);
    float2 bv[NE];
#pragma unroll
    for (int t = 0; t < NE; ++t) bv[t] = cz();
    EC ua[P];
#pragma unroll
    for (int i = 0; i < P; ++i) ua[i] = warm ? sUA[i * RAM] : czero<EC>();

    if (!zero && !bad) {
      double resid = 0.0;
      float anorm2 = 0.f;
#pragma unroll
      for (int e = 0; e < P * P; ++e) anorm2 += cabs2(sA[e]);
      // One LR-Kron half-step pair: the new b = R^T conj(a) / ||a||^2
      // (lane-owned entries, all blocks), then the block pass R conj(b) /
      // ||b||^2 into sAp.  If RES also the residual of (A, b) by the expansion
      // ||R||^2 - 2 Re(a^H R conj(b)) + ||a||^2 ||b||^2, every term summed in
      // FP64 from the FP32 entries (each product exact), so the expansion
      // keeps the residual where it is small.
      auto sweep = [&](bool res) __attribute__((always_inline)) {
        const float ainv = xrcp(anorm2);
        double rr = 0.0, xr = 0.0, b2 = 0.0, a2 = 0.0;
        float bb = 0.f;
        if (res) {
#pragma unroll
          for (int e = 0; e < P * P; ++e) {
            const float2 ae = sA[e];
            a2 = fma(double(ae.x), double(ae.x), fma(double(ae.y), double(ae.y), a2));
          }
        }
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const int e = tid + kWideThreads * t;
          if (e < QQ) {
            // opaque indices: the P^2 entry addresses are formed here, per
            // sweep, not hoisted out of the iteration loop into registers
            int k = e / Q, l = e - (e / Q) * Q;
            asm volatile("" : "+v"(k), "+v"(l));
            float2 bn = cz();
            if (res) {
              // one partial sum per block row: P independent FMA chains
              double px[P], py[P];
#pragma unroll
              for (int i = 0; i < P; ++i) {
                px[i] = 0.0;
                py[i] = 0.0;
#pragma unroll
                for (int j = 0; j < P; ++j) {
                  const float2 sv = Sget(i, j, k, l);
                  const float2 aij = sA[i * P + j];
                  const double ax = aij.x, ay = aij.y, sx = sv.x, sy = sv.y;
                  px[i] = fma(ax, sx, fma(ay, sy, px[i]));
                  py[i] = fma(ax, sy, fma(-ay, sx, py[i]));
                }
              }
              double gx = 0.0, gy = 0.0;
#pragma unroll
              for (int i = 0; i < P; ++i) {
                gx += px[i];
                gy += py[i];
              }
              const double bx = bv[t].x, by = bv[t].y;
              xr = fma(bx, gx, fma(by, gy, xr));
              b2 = fma(bx, bx, fma(by, by, b2));
              bn = make_float2(float(gx) * ainv, float(gy) * ainv);
            } else {
              float2 pb[P];
#pragma unroll
              for (int i = 0; i < P; ++i) {
                pb[i] = cz();
#pragma unroll
                for (int j = 0; j < P; ++j) pb[i] = ccfma(sA[i * P + j], Sget(i, j, k, l), pb[i]);
              }
#pragma unroll
              for (int i = 0; i < P; ++i) bn = cadd(bn, pb[i]);
              bn = cscale(bn, ainv);
            }
            bv[t] = bn;
            bb += cabs2(bn);
            sB[e] = bn;
          } else {
            bv[t] = cz();
          }
        }
        if (res) rr = fma(b2, a2, -2.0 * xr);
        // both sums through one barrier (which also publishes sB); red and
        // redd are next written after the barrier that ends this sweep
        bb = wsum(bb);
        if (res) rr = wsumd(rr);
        if (lane == 0) {
          red[wave] = bb;
          redd[wave] = rr;
        }
        block_sync();
        float bsum = 0.f;
        double rsum = 0.0;
#pragma unroll
        for (int i = 0; i < kWideWaves; ++i) {
          bsum += red[i];
          rsum += redd[i];
        }
        if (res) resid = fmax(normR2 + rsum, 0.0);
        float2 wv[NL];
#pragma unroll
        for (int m = 0; m < NL; ++m) wv[m] = (lane + 64 * m < QQ) ? sB[lane + 64 * m] : cz();
        block_pass(wv, 1.f / bsum, sAp, nullptr);
        block_sync();
      };
      // EIG_{r_a} of Herm(A'), A' = sAp
      auto eig_a = [&](bool cold) __attribute__((always_inline)) {
        if (tid < P * P) {
          const int i = tid / P, j = tid - (tid / P) * P;
          const EC h = cscale(cadd(cto<EC>(sAp[i * P + j]), cconj(cto<EC>(sAp[j * P + i]))), ES(0.5));
          sAh[tid] = h;
        }
        block_sync();
        if (r_a == 1) {
          // wave 0 alone: the iteration is the same on every lane, so the
          // other waves would only take SIMD issue slots from it
          if (wave == 0) {
            if constexpr (PREC == 0) {   // the factor in registers for the iteration (FP32 fits the budget)
              EC mh[P * P];
#pragma unroll
              for (int e = 0; e < P * P; ++e) mh[e] = sAh[e];
              power_top<P, EC>([&](int i, int j) { return mh[i * P + j]; }, ua, cold, 500, 2e-6);
            } else {
              power_top<P, EC>([&](int i, int j) { return sAh[i * P + j]; }, ua, cold, 500, 1e-12);
            }
            ES lam = 0;
#pragma unroll
            for (int i = 0; i < P; ++i) {
              EC s = czero<EC>();
#pragma unroll
              for (int j = 0; j < P; ++j) s = cfma(sAh[i * P + j], ua[j], s);
              lam += ua[i].x * s.x + ua[i].y * s.y;
            }
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
              for (int j = 0; j < P; ++j)
                if (lane == i * P + j) sA[i * P + j] = tof(cscale(cmul(ua[i], cconj(ua[j])), lam));
          }
          block_sync();   // publishes sA; sAh is rewritten by the next call
          anorm2 = 0.f;
#pragma unroll
          for (int e = 0; e < P * P; ++e) anorm2 += cabs2(sA[e]);
          return;
        }
        // r_a > 1: wave 0 runs the subspace iteration with lane k holding row
        // k of Herm(A') and of the basis (dot products by wave reductions),
        // warm-started from the previous U_A; then Hs = U^H Herm(A') U
        // (r_a x r_a) to LDS.  Every thread then forms A = U Hs U^H, with
        // ||A||^2 = ||Hs||_F^2.  The sweep's reduction area is free here and
        // holds the basis exchange and Hs.
        EC* const sVs = reinterpret_cast<EC*>(red);   // [RAM][P] basis exchange
        EC* const sHs = sVs + RAM * P;                 // [RAM][RAM]
        if (wave == 0) {
          const bool rowk = lane < P;
          float2 mrow[P];
#pragma unroll
          for (int j = 0; j < P; ++j) mrow[j] = tof(sAh[(rowk ? lane : 0) * P + j]);
          EC va[RAM];
#pragma unroll
          for (int c = 0; c < RAM; ++c) va[c] = (!cold && rowk) ? sUA[lane * RAM + c] : czero<EC>();
          group_subspace<RAM, 64, P, EC, true>(mrow, rowk, r_a, va, sVs, cold, 500, PREC ? 1e-12 : 2e-6);
          small::lane_sync();
          if (rowk) {
#pragma unroll
            for (int c = 0; c < RAM; ++c)
              if (c < r_a) sUA[lane * RAM + c] = va[c];
          }
          small::lane_sync();
          // (Herm(A') U)[k][b] on lane k, then Hs[a][b] = sum_k conj(U[k][a]) (Herm(A') U)[k][b]
          EC au[RAM];
#pragma unroll
          for (int b = 0; b < RAM; ++b) {
            au[b] = czero<EC>();
            if (b < r_a && rowk) {
#pragma unroll
              for (int j = 0; j < P; ++j) au[b] = cfma(sAh[lane * P + j], sUA[j * RAM + b], au[b]);
            }
          }
#pragma unroll
          for (int a2 = 0; a2 < RAM; ++a2)
#pragma unroll
            for (int b = 0; b < RAM; ++b)
              if (a2 < r_a && b < r_a) {
                const EC hs = gsum<64>(rowk ? ccfma(va[a2], au[b], czero<EC>()) : czero<EC>());
                if (lane == 0) sHs[a2 * RAM + b] = hs;
              }
        }
        block_sync();
        anorm2 = 0.f;
        for (int a2 = 0; a2 < r_a; ++a2)
          for (int b = 0; b < r_a; ++b) anorm2 += float(cabs2(sHs[a2 * RAM + b]));
        if (tid < P * P) {
          const int ai = tid / P, aj = tid - (tid / P) * P;
          EC acc = czero<EC>();
          for (int a2 = 0; a2 < r_a; ++a2) {
            EC t2 = czero<EC>();
            for (int b = 0; b < r_a; ++b) t2 = cfma(sHs[a2 * RAM + b], cconj(sUA[aj * RAM + b]), t2);
            acc = cfma(sUA[ai * RAM + a2], t2, acc);
          }
          sA[tid] = tof(acc);
        }
        block_sync();   // publishes sA; the reduction area is free again
      };
      // sweep 0 has no residual; after sweep k >= 1 the stop rule looks at
      // eta_k (one call site per lambda keeps the code, and its registers, small)
      double eta_prev = INFINITY;
      for (int k = 0;; ++k) {
        sweep(k > 0);
        if (k > 0) {
          const double e = sqrt(resid / normR2);
          eta = float(e);
          const bool stop = iters >= prm.max_iter ||
                            (prm.eps > 0.0 && iters >= prm.min_iter && fabs(e - eta_prev) <= prm.eps);
          if (stop) break;
          eta_prev = e;
        }
        eig_a(k == 0 && !warm);
        iters = k + 1;
      }
    }
    // U_A of this pixel (rows of the r_a = 1 power iterate, or the subspace)
    block_sync();
    if (tid == 0 && r_a == 1) {
#pragma unroll
      for (int i = 0; i < P; ++i) sUA[i * RAM] = ua[i];
    }
    chain = !bad;   // this S may seed the next pixel's
    ua_ok = !zero && !bad;
    block_sync();
    // ------------------------------------------ enqueue for the batched tail
    // (sB holds the final b = R^T conj(a) / ||a||^2 of a finite pixel)
    float2* const hq = sHq + nq * QQ;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tid + kWideThreads * t;
      if (e < QQ) {
        const int k = e / Q, l = e - (e / Q) * Q;
        hq[e] = cscale(cadd(sB[k * Q + l], cconj(sB[l * Q + k])), 0.5f);
      }
    }
    if (tid == 0) {
      sQidx[nq] = idx;
      sQflag[nq] = bad ? 2 : (zero ? 1 : 0);
      sQeta[nq] = eta;
      sQit[nq] = iters;
    }
    if (tid < P * RAM) sQUA[nq][tid] = (zero || bad) ? czero<EC>() : sUA[tid];
    block_sync();
    ++nq;
  };

  // one call site each for the pixel body and the tail
  for (int64_t itp = 0;; ++itp) {
    const bool more = itp < count;
    if (more) pixel(itp);
    if (nq == NQ || (!more && nq > 0)) {
      tail(nq);
      nq = 0;
    }
    if (!more) break;
  }
}

template <int P, int Q, int RBM, int MODE, int PREC, bool VAR = false>
__global__ __launch_bounds__(kWideThreads, 1) void kstap_wide_kernel(const KParams prm) {
  __shared__ __attribute__((aligned(16))) char lds[WideLds<P, Q, RBM, PREC>::bytes];
  int64_t first, count;
  if (MODE == kModeRun) {
    const int per = gridDim.x >> 3;
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (logical >= prm.nlogical) return;
    const int64_t total = tiled_positions(prm.H, prm.W);
    first = int64_t(logical) * prm.pix_per_block;
    count = total - first;
    if (count > prm.pix_per_block) count = prm.pix_per_block;
  } else {
    first = int64_t(blockIdx.x) * prm.pix_per_block;
    count = prm.npix - first;
    if (count > prm.pix_per_block) count = prm.pix_per_block;
  }
  run_pixels_wide<P, Q, RBM, MODE, PREC, VAR>(prm, first, count, lds);
}

// ---------------------------------------------------------------- launchers
template <int P, int Q, int RBM, int PREC>
int launch_one(int mode, const KParams& prm, hipStream_t stream) {
  int64_t units = (mode == kModeRun) ? int64_t(prm.nlogical) : (int64_t(prm.npix) + prm.pix_per_block - 1) / prm.pix_per_block;
  if (units <= 0) return hipSuccess;
  int64_t grid = (mode == kModeRun) ? ((units + 7) / 8) * 8 : units;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (mode == kModeRun && has_variants(prm))
    hipLaunchKernelGGL((kstap_kernel<P, Q, RBM, kModeRun, PREC, true>), dim3(unsigned(grid)), dim3(64), 0, stream,
                       prm);
  else if (mode == kModeRun)
    hipLaunchKernelGGL((kstap_kernel<P, Q, RBM, kModeRun, PREC>), dim3(unsigned(grid)), dim3(64), 0, stream, prm);
  else
    hipLaunchKernelGGL((kstap_kernel<P, Q, RBM, kModeProbe, PREC>), dim3(unsigned(grid)), dim3(64), 0, stream, prm);
  return hipGetLastError();
}

template <int P, int Q, int RBM, int PREC>
int launch_wide(int mode, const KParams& prm, hipStream_t stream) {
  int64_t units = (mode == kModeRun) ? int64_t(prm.nlogical) : (int64_t(prm.npix) + prm.pix_per_block - 1) / prm.pix_per_block;
  if (units <= 0) return hipSuccess;
  int64_t grid = (mode == kModeRun) ? ((units + 7) / 8) * 8 : units;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (mode == kModeRun && has_variants(prm))
    hipLaunchKernelGGL((kstap_wide_kernel<P, Q, RBM, kModeRun, PREC, true>), dim3(unsigned(grid)), dim3(kWideThreads), 0,
                       stream, prm);
  else if (mode == kModeRun)
    hipLaunchKernelGGL((kstap_wide_kernel<P, Q, RBM, kModeRun, PREC>), dim3(unsigned(grid)), dim3(kWideThreads), 0, stream,
                       prm);
  else
    hipLaunchKernelGGL((kstap_wide_kernel<P, Q, RBM, kModeProbe, PREC>), dim3(unsigned(grid)), dim3(kWideThreads), 0, stream,
                       prm);
  return hipGetLastError();
}

template <int P, int Q, int RBM, int PREC>
int launch_persist(const KParams* descs, const int32_t* order, const int64_t* prefix, int nt, int ppb,
                   unsigned long long* counter, int grid, hipStream_t stream) {
  hipLaunchKernelGGL((kstap_persistent<P, Q, RBM, PREC>), dim3(grid), dim3(64), 0, stream, descs, order, prefix, nt,
                     ppb, counter);
  return hipGetLastError();
}

}  // namespace
}  // namespace kstap
