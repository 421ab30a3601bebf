// Small dense complex FP64 helpers shared by the single-covariance and
// LR-STAP kernels: complex arithmetic, wave reductions, and the Jacobi
// eigen-decomposition of a Hermitian matrix of order <= 8 in parallel order
// with one lane per matrix entry.
#pragma once

#include <hip/hip_runtime.h>

namespace kstap {
namespace small {

struct dc {
  double x, y;
};
__device__ __forceinline__ dc mk(double x, double y) { return dc{x, y}; }
__device__ __forceinline__ dc add(dc a, dc b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ dc sub(dc a, dc b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ dc mul(dc a, dc b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ dc cj(dc a) { return mk(a.x, -a.y); }
__device__ __forceinline__ dc scl(dc a, double s) { return mk(a.x * s, a.y * s); }
__device__ __forceinline__ double ab2(dc a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 64 lanes by DPP row reductions and row broadcasts (no LDS
// traffic); every lane must be active.  The total is read from lane 63.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const int2 i = __builtin_bit_cast(int2, v);
  int2 o;
  o.x = __builtin_amdgcn_update_dpp(0, i.x, CTRL, ROWS, 0xF, false);
  o.y = __builtin_amdgcn_update_dpp(0, i.y, CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, o);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_d<0x140, 0xF>(v);   // row_mirror
  v += dpp_d<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  const int2 i = __builtin_bit_cast(int2, v);
  int2 o;
  o.x = __builtin_amdgcn_readlane(i.x, 63);
  o.y = __builtin_amdgcn_readlane(i.y, 63);
  return __builtin_bit_cast(double, o);
}

// Wave-local LDS exchange: a wavefront's LDS operations complete in issue
// order, so only the compiler has to be kept from moving accesses across.
__device__ __forceinline__ void lane_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Partner of index k in round s of the circle schedule over PE (even)
// indices: index 0 stays, the others rotate, position t meets position
// PE - 1 - t.  Over PE - 1 rounds every pair meets once.
__device__ __forceinline__ int rr_partner(int k, int s, int PE) {
  const int m = PE - 1;
  const int pos = (k == 0) ? 0 : 1 + ((k - 1 - s) % m + m) % m;
  const int t = PE - 1 - pos;
  return (t == 0) ? 0 : 1 + (t - 1 + s) % m;
}

__device__ __forceinline__ dc shd(dc x, int src) { return mk(__shfl(x.x, src, 64), __shfl(x.y, src, 64)); }

// Eigen-decomposition of a Hermitian P x P matrix by Jacobi rotations in
// parallel order, run by one wavefront with one lane per matrix entry: lane
// r PE + c holds h = H[r][c] and v = V[r][c] (PE = P rounded up to even; a
// zero pad row and column when P is odd, which no rotation touches).  Each
// round applies PE / 2 rotations on disjoint index pairs at once, and each
// rotation U = D [c s; -s c] on the pair (a, b), a < b, D = diag(1, e^{-i phi})
// making H[a][b] real, zeroes H[a][b]: H <- U^H H U, V <- V U.  On return the
// diagonal lanes hold the eigenvalues (unsorted) and V the eigenvectors as
// columns.
__device__ __forceinline__ void jacobi_par_n(dc& h, dc& v, int lane, const int P) {
  const int PE = (P + 1) / 2 * 2;
  const bool in = lane < PE * PE;
  const int r = in ? lane / PE : 0, c = in ? lane - (lane / PE) * PE : 0;
  v = mk((in && r == c) ? 1.0 : 0.0, 0.0);
  if (!in) h = mk(0, 0);
  for (int sweep = 0; sweep < 30; ++sweep) {
    const double m2 = ab2(h);
    const double off = wave_sum(r != c ? m2 : 0.0), tot = wave_sum(m2);
    if (off <= 1e-30 * tot) break;   // uniform
    const double small = 1e-300 * sqrt(tot);
    for (int s = 0; s < PE - 1; ++s) {
      // U[k][k] (us) and U[partner][k] (uo) of the rotation that holds index k
      auto params = [&](int k, int kp, dc& us, dc& uo) {
        const int a = min(k, kp), b = max(k, kp);
        const dc hab = shd(h, a * PE + b);
        const double haa = shd(h, a * PE + a).x, hbb = shd(h, b * PE + b).x;
        const double rr = sqrt(ab2(hab));
        if (rr <= small) {
          us = mk(1, 0);
          uo = mk(0, 0);
          return;
        }
        const dc e = scl(hab, 1.0 / rr);   // e^{i phi}
        const double tau = (hbb - haa) / (2.0 * rr);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
        if (k == a) {   // column a of U: (c, -s conj(e))
          us = mk(cs, 0);
          uo = scl(cj(e), -sn);
        } else {        // column b of U: (s, c conj(e))
          us = scl(cj(e), cs);
          uo = mk(sn, 0);
        }
      };
      const int rp = rr_partner(r, s, PE), cp = rr_partner(c, s, PE);
      dc usr, uor, usc, uoc;
      params(r, rp, usr, uor);
      params(c, cp, usc, uoc);
      const dc h_rcp = shd(h, r * PE + cp), h_rpc = shd(h, rp * PE + c), h_rpcp = shd(h, rp * PE + cp);
      const dc v_rcp = shd(v, r * PE + cp);
      // H'[r][c] = sum over s in {r, r'}, t in {c, c'} of conj(U[s][r]) H[s][t] U[t][c]
      const dc t1 = add(mul(h, usc), mul(h_rcp, uoc));
      const dc t2 = add(mul(h_rpc, usc), mul(h_rpcp, uoc));
      dc hn = add(mul(cj(usr), t1), mul(cj(uor), t2));
      const dc vn = add(mul(v, usc), mul(v_rcp, uoc));
      if (r != c && c == rp) hn = mk(0, 0);   // the rotated pair's off-diagonal entries
      if (r == c) hn.y = 0;
      h = in ? hn : mk(0, 0);
      v = in ? vn : mk(0, 0);
    }
  }
}

// Order P fixed at compile time.
template <int P>
__device__ __forceinline__ void jacobi_par(dc& h, dc& v, int lane) {
  jacobi_par_n(h, v, lane, P);
}

}  // namespace small
}  // namespace kstap
