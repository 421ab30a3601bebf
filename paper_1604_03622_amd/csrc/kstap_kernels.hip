// Fused per-pixel Kronecker STAP kernels for gfx950 (MI355X).
//
// One 64-lane wavefront (one workgroup) carries one pixel at a time through
// the whole pass; a workgroup walks a run of consecutive pixels of a row.
//
//   a2  sample covariance S = (1/n) sum_m x_m x_m^H  (Sec. 1.1, Eq. (2)) as a
//       dense contraction on FP32 MFMA (v_mfma_f32_16x16x4_f32).  With
//       Y = [Re x; Im x] the real Gram has the blocks Re S = Xr Xr^T + Xi Xi^T
//       and Im S = Xi Xr^T - Xr Xi^T; only the upper 16 x 16 tiles are formed,
//       and the diagonal tiles of Im S use one product and its transpose.
//       Operands come straight from global memory (neighbouring pixels of a
//       workgroup, and the workgroups of one XCD, share them through L1/L2).
//   a3  the rearrangement of Algorithm 1 is never materialised: block S(i,j)
//       of S is row i*p + j... of R in address arithmetic only.
//   a4  A_0 = block sums of S / q^2 (Sec. 4, Eqs. (18)-(19)).
//   a5  LR-Kron (Algorithm 2) on the LDS-resident S: one sweep over S per
//       iteration computes the residual of the previous iterate, the new time
//       factor b = R^T conj(a) / ||a||^2 and the partial sums of R conj(b).
//       EIG_{r_a} (Eq. (17)) by subspace iteration with a warm start.
//   a6  final b = R^T conj(a) / ||a||^2, Hermitian part, top-r_b subspace by
//       subspace iteration (CholQR2 orthonormalisation, residual stop).
//   a8  T = ||F_A X conj(F_B b_s)||^2 / (b_s^H F_B b_s) (Sec. 5, Eq. (25);
//       Sec. 6.3, Eq. (26)); D = T > tau.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kstap_internal.h"

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

// ------------------------------------------------------- wavefront reductions
// Sum over the 64 lanes, result in every lane: four DPP steps inside each
// 16-lane row (quad swaps, half-row mirror, row mirror), then two lane
// permutes across rows.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wsum(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ __forceinline__ float2 wsum(float2 v) { return make_float2(wsum(v.x), wsum(v.y)); }
__device__ __forceinline__ double wsumd(double v) {
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }   // one-wave workgroups

__device__ __forceinline__ float frac01(float x) { return x - floorf(x); }

// Deterministic, generic start block for subspace iteration.
__device__ __forceinline__ float2 omega(int k, int c) {
  float ph = 6.2831853f * frac01(0.6180340f * (k + 1) + 0.4142136f * (c + 1) * (k + 3));
  return make_float2(__cosf(ph), __sinf(ph));
}

// ------------------------------------------------- small Hermitian subspaces
// Orthonormalise the rows held by the lanes (lane k < d holds row k of a
// d x r block W) by Cholesky QR: G = W^H W = L L^H, V = W L^{-H}.
template <int RM>
__device__ __forceinline__ void chol_qr(float2 (&w)[RM], int r, bool act) {
  float2 G[RM][RM];
#pragma unroll
  for (int a = 0; a < RM; ++a)
#pragma unroll
    for (int b = a; b < RM; ++b) {
      if (a < r && b < r) {
        float2 g = act ? ccfma(w[a], w[b], cz()) : cz();
        G[a][b] = wsum(g);
      } else {
        G[a][b] = cz();
      }
    }
  float2 L[RM][RM];
  float dinv[RM];
  float tr = 0.f;
#pragma unroll
  for (int a = 0; a < RM; ++a) tr += (a < r) ? G[a][a].x : 0.f;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    if (j >= r) { dinv[j] = 0.f; continue; }
    float dj = G[j][j].x;
#pragma unroll
    for (int a = 0; a < j; ++a) dj -= cabs2(L[j][a]);
    dj = fmaxf(dj, 1e-30f + 1e-14f * tr);
    const float ljj = sqrtf(dj);
    dinv[j] = 1.f / ljj;
    L[j][j] = make_float2(ljj, 0.f);
#pragma unroll
    for (int i = j + 1; i < RM; ++i) {
      if (i >= r) continue;
      float2 s = cconj(G[j][i]);   // G[i][j]
#pragma unroll
      for (int a = 0; a < j; ++a) s = csub(s, cmul(L[i][a], cconj(L[j][a])));
      L[i][j] = cscale(s, dinv[j]);
    }
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      if (c >= r) continue;
      float2 s = w[c];
#pragma unroll
      for (int a = 0; a < c; ++a) s = csub(s, cmul(w[a], cconj(L[c][a])));
      w[c] = cscale(s, dinv[c]);
    }
  }
}

// Top-r invariant subspace of the Hermitian d x d matrix M (LDS, row-major)
// by subspace iteration.  Lane k < d holds row k of the orthonormal basis v.
// `cold` starts from M * Omega; otherwise v is the warm start.  Stops `extra`
// steps after ||M V - V (V^H M V)||_F <= tol ||M V||_F, or after max_steps.
template <int RM>
__device__ int top_subspace(const float2* M, int d, int r, float2 (&v)[RM], float2* sV,
                            bool cold, int max_steps, float tol, int extra) {
  const int k = threadIdx.x;
  const bool act = k < d;
  if (cold) {
#pragma unroll
    for (int c = 0; c < RM; ++c) v[c] = (act && c < r) ? omega(k, c) : cz();
  }
  bool ortho = !cold;
  int step = 0, after = -1;
  while (true) {
    if (act) {
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < r) sV[c * d + k] = v[c];
    }
    wave_sync();
    float2 w[RM];
#pragma unroll
    for (int c = 0; c < RM; ++c) w[c] = cz();
    if (act) {
      for (int l = 0; l < d; ++l) {
        const float2 m = M[k * d + l];
#pragma unroll
        for (int c = 0; c < RM; ++c)
          if (c < r) w[c] = cfma(m, sV[c * d + l], w[c]);
      }
    }
    wave_sync();
    bool conv = false;
    if (ortho) {
      // H = V^H W (Hermitian), residual W - V H
      float2 Hm[RM][RM];
#pragma unroll
      for (int a = 0; a < RM; ++a)
#pragma unroll
        for (int b = a; b < RM; ++b) {
          if (a < r && b < r) {
            Hm[a][b] = wsum(act ? ccfma(v[a], w[b], cz()) : cz());
            Hm[b][a] = cconj(Hm[a][b]);
          }
        }
      float rn = 0.f, wn = 0.f;
      if (act) {
#pragma unroll
        for (int b = 0; b < RM; ++b) {
          if (b >= r) continue;
          float2 rr = w[b];
#pragma unroll
          for (int a = 0; a < RM; ++a)
            if (a < r) rr = csub(rr, cmul(v[a], Hm[a][b]));
          rn += cabs2(rr);
          wn += cabs2(w[b]);
        }
      }
      rn = wsum(rn);
      wn = wsum(wn);
      conv = rn <= tol * tol * wn;
    }
    chol_qr<RM>(w, r, act);
    chol_qr<RM>(w, r, act);
#pragma unroll
    for (int c = 0; c < RM; ++c) v[c] = w[c];
    ortho = true;
    ++step;
    if (conv && after < 0) after = 0;
    if (after >= 0) {
      if (after >= extra) break;
      ++after;
    }
    if (step >= max_steps) break;
  }
  return step;
}

// ------------------------------------------------------------ kernel body
template <int P, int Q, int RBM, int MODE>
__global__ __launch_bounds__(64) void kstap_fp32_kernel(const KParams prm) {
  constexpr int PQ = P * Q;
  constexpr int NB = (PQ + 15) / 16;        // 16-row blocks of the pq x pq covariance
  constexpr int NT = NB * (NB + 1) / 2;     // upper tiles of Re S
  constexpr int NO = NB * (NB - 1) / 2;     // strictly upper tiles of Im S
  constexpr int QQ = Q * Q;
  constexpr int NE = (QQ + 63) / 64;        // q x q entries per lane
  constexpr int RAM = (P < kMaxRA) ? P : kMaxRA;
  static_assert(PQ * PQ >= 2 * QQ + RBM * Q, "LDS reuse needs p >= 2");

  __shared__ float2 sS[PQ * PQ];
  __shared__ int sOff[kMaxN];
  __shared__ float2 sA[P * P];
  __shared__ float2 sUA[P * RAM];
  __shared__ float2 sVa[P * RAM];

  const int lane = threadIdx.x;
  const int n = prm.n;
  const int H = prm.H, W = prm.W;
  const int r_a = prm.r_a, r_b = prm.r_b;

  for (int m = lane; m < n; m += 64) sOff[m] = (int(prm.st[2 * m]) * W + int(prm.st[2 * m + 1])) * Q;
  wave_sync();

  // Operand rows of this lane: row rho = 16*I + (lane & 15) of the stacked
  // snapshot, channel rho / q, sample rho % q.
  int chan_off[NB];
  bool row_ok[NB];
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    const int rho = 16 * I + (lane & 15);
    row_ok[I] = rho < PQ;
    const int ch = rho / Q, j = rho - ch * Q;
    chan_off[I] = row_ok[I] ? ch * H * W * Q + j : 0;
  }

  // pixel schedule
  int64_t first, count;
  if (MODE == kModeRun) {
    const int per = gridDim.x >> 3;   // grid is a multiple of 8 (one share per XCD)
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (logical >= prm.nlogical) return;
    const int64_t total = int64_t(H) * W;
    first = int64_t(logical) * prm.pix_per_block;
    count = total - first;
    if (count > prm.pix_per_block) count = prm.pix_per_block;
  } else {
    first = int64_t(blockIdx.x) * prm.pix_per_block;
    count = prm.npix - first;
    if (count > prm.pix_per_block) count = prm.pix_per_block;
  }

  for (int64_t it = 0; it < count; ++it) {
    const int64_t idx = first + it;
    int r, c;
    if (MODE == kModeRun) {
      r = int(idx / W);
      c = int(idx - int64_t(r) * W);
    } else {
      r = prm.pix[2 * idx];
      c = prm.pix[2 * idx + 1];
    }
    const bool valid = r >= prm.r0 && r < prm.r1 && c >= prm.c0 && c < prm.c1;
    const int64_t out_idx = idx;
    if (!valid) {
      if (lane == 0) {
        prm.T[out_idx] = 0.f;
        if (MODE == kModeRun && prm.D) prm.D[out_idx] = 0;
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
    const float2* xp = prm.x + (int64_t(r) * W + c) * Q;

    // ---------------------------------------------------------------- a2 SCM
    f4 accR[NT], accI[NO > 0 ? NO : 1], accD[NB];
#pragma unroll
    for (int t = 0; t < NT; ++t) accR[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < (NO > 0 ? NO : 1); ++t) accI[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NB; ++t) accD[t] = f4{0.f, 0.f, 0.f, 0.f};

    const int nch = (n + 3) >> 2;
    float2 cur[NB], nxt[NB];
    {
      const int m = lane >> 4;
      const bool mok = m < n;
      const int off = sOff[mok ? m : 0];
#pragma unroll
      for (int I = 0; I < NB; ++I) cur[I] = (mok && row_ok[I]) ? xp[chan_off[I] + off] : cz();
    }
    for (int ch = 0; ch < nch; ++ch) {
      {
        const int m = (ch + 1) * 4 + (lane >> 4);
        const bool mok = m < n;
        const int off = sOff[mok ? m : 0];
#pragma unroll
        for (int I = 0; I < NB; ++I) nxt[I] = (mok && row_ok[I]) ? xp[chan_off[I] + off] : cz();
      }
      float xr[NB], xi[NB], nxr[NB];
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        xr[I] = cur[I].x;
        xi[I] = cur[I].y;
        nxr[I] = -cur[I].x;
      }
      int t = 0, u = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int J = I; J < NB; ++J) {
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[I], xr[J], accR[t], 0, 0, 0);
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[I], xi[J], accR[t], 0, 0, 0);
          if (J > I) {
            accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[I], xr[J], accI[u], 0, 0, 0);
            accI[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(nxr[I], xi[J], accI[u], 0, 0, 0);
            ++u;
          } else {
            accD[I] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[I], xr[I], accD[I], 0, 0, 0);
          }
          ++t;
        }
      }
#pragma unroll
      for (int I = 0; I < NB; ++I) cur[I] = nxt[I];
    }

    // S to LDS, full Hermitian, scaled by 1/n.  MFMA output layout: lane l,
    // register q holds row 4*(l/16) + q, column l % 16 of the 16 x 16 tile.
    const float inv_n = 1.f / float(n);
    const int trow = 4 * (lane >> 4), tcol = lane & 15;
    {
      int t = 0, u = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I) {
#pragma unroll
        for (int J = I; J < NB; ++J) {
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            const int row = 16 * I + trow + q4, col = 16 * J + tcol;
            if (row < PQ && col < PQ) {
              const float re = accR[t][q4] * inv_n;
              if (J > I) {
                const float im = accI[u][q4] * inv_n;
                sS[row * PQ + col] = make_float2(re, im);
                sS[col * PQ + row] = make_float2(re, -im);
              } else {
                sS[row * PQ + col] = make_float2(re, accD[I][q4] * inv_n);
              }
            }
          }
          if (J > I) ++u;
          ++t;
        }
      }
    }
    wave_sync();
    {
      float tr_[NB][4];
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int row = 16 * I + trow + q4, col = 16 * I + tcol;
          tr_[I][q4] = (row < PQ && col < PQ) ? sS[col * PQ + row].y : 0.f;
        }
      wave_sync();
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int row = 16 * I + trow + q4, col = 16 * I + tcol;
          if (row < PQ && col < PQ) sS[row * PQ + col].y = accD[I][q4] * inv_n - tr_[I][q4];
        }
    }
    wave_sync();

    // ------------------------------------------------ a4 init, ||R||_F = ||S||_F
    float2 A[P * P];
    double normR2;
    {
      float2 a0[P * P], pt[P * P];
#pragma unroll
      for (int e = 0; e < P * P; ++e) a0[e] = pt[e] = cz();
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
              const float2 s = sS[(i * Q + k) * PQ + j * Q + l];
              a0[i * P + j] = cadd(a0[i * P + j], s);
              if (k == l) pt[i * P + j] = cadd(pt[i * P + j], s);
              nr += cabs2(s);
            }
        }
      }
      normR2 = wsumd(double(nr));
      float an = 0.f;
#pragma unroll
      for (int e = 0; e < P * P; ++e) {
        a0[e] = cscale(wsum(a0[e]), 1.f / float(QQ));
        an += cabs2(a0[e]);
      }
      const bool fallback = double(an) <= 1e-24 * normR2;
#pragma unroll
      for (int e = 0; e < P * P; ++e) A[e] = fallback ? wsum(pt[e]) : a0[e];
    }

    float T = 0.f, eta = 0.f;
    int iters = 0;
    const bool zero = !(normR2 > 0.0);
    const bool bad = !isfinite(normR2);
    float2 va[RAM];
    float2 vb[RBM];
#pragma unroll
    for (int c = 0; c < RAM; ++c) va[c] = cz();
#pragma unroll
    for (int c = 0; c < RBM; ++c) vb[c] = cz();

    if (!zero && !bad) {
      // --------------------------------------------------------- a5 LR-Kron
      float2 bv[NE];
      float2 Ap[P * P];
      float bn2;
      double resid = 0.0;
      float anorm2 = 0.f;
#pragma unroll
      for (int e = 0; e < P * P; ++e) anorm2 += cabs2(A[e]);

      // one sweep over S: residual of (A, bv) if RES, then the new b and the
      // partial sums of R conj(b)
      auto sweep = [&](bool res) {
        const float ainv = 1.f / anorm2;
        float2 ap[P * P];
#pragma unroll
        for (int e = 0; e < P * P; ++e) ap[e] = cz();
        float bb = 0.f;
        double rr = 0.0;
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const int e = lane + 64 * t;
          if (e < QQ) {
            const int k = e / Q, l = e - (e / Q) * Q;
            float2 s[P * P];
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
              for (int j = 0; j < P; ++j) s[i * P + j] = sS[(i * Q + k) * PQ + j * Q + l];
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
        bn2 = wsum(bb);
        const float binv = 1.f / bn2;
#pragma unroll
        for (int ij = 0; ij < P * P; ++ij) Ap[ij] = cscale(wsum(ap[ij]), binv);
        if (res) resid = wsumd(rr);
      };

      // EIG_{r_a}: A <- U (U^H A' U) U^H with U the top-r_a subspace of Herm(A')
      auto eig_a = [&](bool cold) {
        if (lane == 0) {
#pragma unroll
          for (int i = 0; i < P; ++i)
#pragma unroll
            for (int j = 0; j < P; ++j)
              sA[i * P + j] = cscale(cadd(Ap[i * P + j], cconj(Ap[j * P + i])), 0.5f);
        }
        wave_sync();
        top_subspace<RAM>(sA, P, r_a, va, sVa, cold, 200, 2e-6f, 1);
        if (lane < P) {
#pragma unroll
          for (int c = 0; c < RAM; ++c)
            if (c < r_a) sUA[lane * RAM + c] = va[c];
        }
        wave_sync();
        float2 U[P][RAM];
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
          for (int c = 0; c < RAM; ++c) U[i][c] = (c < r_a) ? sUA[i * RAM + c] : cz();
        // Hs = U^H Herm(A') U
        float2 Hs[RAM][RAM];
#pragma unroll
        for (int a = 0; a < RAM; ++a)
#pragma unroll
          for (int b = 0; b < RAM; ++b) {
            float2 s = cz();
            if (a < r_a && b < r_a) {
#pragma unroll
              for (int i = 0; i < P; ++i) {
                float2 t2 = cz();
#pragma unroll
                for (int j = 0; j < P; ++j) t2 = cfma(sA[i * P + j], U[j][b], t2);
                s = ccfma(U[i][a], t2, s);
              }
            }
            Hs[a][b] = s;
          }
        anorm2 = 0.f;
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
          for (int j = 0; j < P; ++j) {
            float2 s = cz();
#pragma unroll
            for (int a = 0; a < RAM; ++a)
#pragma unroll
              for (int b = 0; b < RAM; ++b)
                if (a < r_a && b < r_a) s = cfma(cmul(U[i][a], Hs[a][b]), cconj(U[j][b]), s);
            A[i * P + j] = s;
            anorm2 += cabs2(s);
          }
        wave_sync();
      };

      sweep(false);
      eig_a(true);
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

      // --------------------------------------------- a6 temporal subspace
      wave_sync();   // S is dead from here on
      float2* sB = sS;          // raw B, row-major q x q (B[k][l] = b[k + q l] in vec form)
      float2* sBh = sS + QQ;    // Hermitian part
      float2* sVb = sS + 2 * QQ;
#pragma unroll
      for (int t = 0; t < NE; ++t) {
        const int e = lane + 64 * t;
        if (e < QQ) sB[e] = bv[t];
      }
      wave_sync();
#pragma unroll
      for (int t = 0; t < NE; ++t) {
        const int e = lane + 64 * t;
        if (e < QQ) {
          const int k = e / Q, l = e - (e / Q) * Q;
          sBh[e] = cscale(cadd(sB[k * Q + l], cconj(sB[l * Q + k])), 0.5f);
        }
      }
      wave_sync();
      if (r_b > 0) top_subspace<RBM>(sBh, Q, r_b, vb, sVb, true, 200, 2e-6f, 1);

      // ------------------------------------------------------ a8 statistic
      const int k = lane;
      const bool kq = k < Q;
      const float2 bsk = kq ? prm.b_s[k] : cz();
      float2 g = bsk;
      if (r_b > 0) {
        float2 coef[RBM];
#pragma unroll
        for (int c = 0; c < RBM; ++c)
          if (c < r_b) coef[c] = wsum(kq ? ccfma(vb[c], bsk, cz()) : cz());
        if (kq) {
#pragma unroll
          for (int c = 0; c < RBM; ++c)
            if (c < r_b) g = csub(g, cmul(vb[c], coef[c]));
        }
      }
      float2 w[P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const float2 xv = kq ? xp[int64_t(i) * H * W * Q + k] : cz();
        w[i] = wsum(kq ? cmul(xv, cconj(g)) : cz());
      }
      const float den = wsum(kq ? fmaf(bsk.x, g.x, bsk.y * g.y) : 0.f);
      // z = F_A w with U_A from the last EIG (sUA)
      float2 U[P][RAM];
#pragma unroll
      for (int i = 0; i < P; ++i)
#pragma unroll
        for (int c = 0; c < RAM; ++c) U[i][c] = (c < r_a) ? sUA[i * RAM + c] : cz();
      float2 z[P];
      {
        float2 cw[RAM];
#pragma unroll
        for (int c = 0; c < RAM; ++c) {
          cw[c] = cz();
          if (c < r_a) {
#pragma unroll
            for (int i = 0; i < P; ++i) cw[c] = ccfma(U[i][c], w[i], cw[c]);
          }
        }
#pragma unroll
        for (int i = 0; i < P; ++i) {
          z[i] = w[i];
#pragma unroll
          for (int c = 0; c < RAM; ++c)
            if (c < r_a) z[i] = csub(z[i], cmul(U[i][c], cw[c]));
        }
      }
      const bool den_ok = den > 1e-12f * prm.bs_norm2;
      if (prm.stat_mode == 0) {
        float num = 0.f;
#pragma unroll
        for (int i = 0; i < P; ++i) num += cabs2(z[i]);
        T = den_ok ? num / den : 0.f;
      } else {
        float2 hz = cz(), fh[P];
#pragma unroll
        for (int i = 0; i < P; ++i) fh[i] = prm.h_s[i];
#pragma unroll
        for (int c = 0; c < RAM; ++c) {
          if (c >= r_a) continue;
          float2 ch = cz();
#pragma unroll
          for (int i = 0; i < P; ++i) ch = ccfma(U[i][c], prm.h_s[i], ch);
#pragma unroll
          for (int i = 0; i < P; ++i) fh[i] = csub(fh[i], cmul(U[i][c], ch));
        }
        float hfh = 0.f;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          hz = ccfma(prm.h_s[i], z[i], hz);
          hfh += fmaf(prm.h_s[i].x, fh[i].x, prm.h_s[i].y * fh[i].y);
        }
        const bool ok = den_ok && hfh > 1e-12f * prm.h_norm2;
        T = ok ? cabs2(hz) / (hfh * den) : 0.f;
      }
      if (!isfinite(T)) T = NAN;
    } else if (bad) {
      T = NAN;
    }

    if (lane == 0) {
      prm.T[out_idx] = T;
      if (MODE == kModeRun && prm.D) prm.D[out_idx] = (T > prm.tau) ? 1 : 0;
      if (MODE == kModeProbe) {
        if (prm.eta) prm.eta[idx] = eta;
        if (prm.iters) prm.iters[idx] = iters;
      }
    }
    if (MODE == kModeProbe) {
      if (prm.UA && lane < P) {
#pragma unroll
        for (int c = 0; c < RAM; ++c)
          if (c < r_a) prm.UA[(idx * P + lane) * r_a + c] = (zero || bad) ? cz() : sUA[lane * RAM + c];
      }
      if (prm.UB && lane < Q) {
#pragma unroll
        for (int c = 0; c < RBM; ++c)
          if (c < r_b) prm.UB[(idx * Q + lane) * r_b + c] = (zero || bad) ? cz() : vb[c];
      }
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- dispatch
typedef void (*KernelFn)(const KParams);

template <int P, int Q, int RBM>
int launch_one(int mode, const KParams& prm, hipStream_t stream) {
  int64_t units = (mode == kModeRun) ? int64_t(prm.nlogical) : (int64_t(prm.npix) + prm.pix_per_block - 1) / prm.pix_per_block;
  if (units <= 0) return hipSuccess;
  int64_t grid = (mode == kModeRun) ? ((units + 7) / 8) * 8 : units;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (mode == kModeRun)
    hipLaunchKernelGGL((kstap_fp32_kernel<P, Q, RBM, kModeRun>), dim3(unsigned(grid)), dim3(64), 0, stream, prm);
  else
    hipLaunchKernelGGL((kstap_fp32_kernel<P, Q, RBM, kModeProbe>), dim3(unsigned(grid)), dim3(64), 0, stream, prm);
  return hipGetLastError();
}

struct Entry {
  int p, q, rbm;
  int (*fn)(int, const KParams&, hipStream_t);
};

#define KSTAP_ENTRY(P, Q, R) {P, Q, R, &launch_one<P, Q, R>}
const Entry kTable[] = {
    KSTAP_ENTRY(2, 8, 4),  KSTAP_ENTRY(2, 16, 4), KSTAP_ENTRY(2, 32, 4),
    KSTAP_ENTRY(3, 8, 4),  KSTAP_ENTRY(3, 8, 8),  KSTAP_ENTRY(3, 12, 4), KSTAP_ENTRY(3, 12, 8),
    KSTAP_ENTRY(3, 16, 4), KSTAP_ENTRY(3, 16, 8), KSTAP_ENTRY(4, 8, 4),  KSTAP_ENTRY(4, 16, 4),
    KSTAP_ENTRY(6, 8, 4),
};
#undef KSTAP_ENTRY

const Entry* find(int p, int q, int r_b) {
  const int rbm = (r_b <= 4) ? 4 : 8;
  for (const Entry& e : kTable)
    if (e.p == p && e.q == q && e.rbm == rbm) return &e;
  return nullptr;
}

}  // namespace

bool kernel_available(int p, int q, int r_b, int precision) {
  if (precision != 0) return false;
  return find(p, q, r_b) != nullptr;
}

int launch_pixels(int p, int q, int precision, int mode, const KParams& prm, hipStream_t stream) {
  if (precision != 0) return hipErrorInvalidValue;
  const Entry* e = find(p, q, prm.r_b);
  if (!e) return hipErrorInvalidValue;
  return e->fn(mode, prm, stream);
}

}  // namespace kstap
