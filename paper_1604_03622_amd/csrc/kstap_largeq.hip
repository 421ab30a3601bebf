// LR-Kron on one large covariance (Sec. 6.1: p channels, q up to thousands of
// azimuth samples, a few training snapshots), without forming S or R.
//
// For S = (1/n) sum_m x_m x_m^H with x_m = vec(X_m^T) (Eq. (2)), Algorithm 1
// maps every rank-one term to a Kronecker product of the snapshot with its
// conjugate: R(x_m x_m^H)[a p + b][l q + k] = conj(X_m[a][l]) X_m[b][k], so
// R(S) = (1/n) sum_m conj(X_m) (x) X_m.  Both half-steps of Algorithm 2 then
// reduce to p x p algebra on the n^2 Gram blocks G_mm' = X_m X_m'^H:
//   B = c sum_m X_m^T conj(A) conj(X_m),  c = 1 / (n ||A||^2)
//   R conj(b) = c sum_{m,m'} G_m'm A G_mm'
//   ||b||^2 = c^2 Re sum_{m,m'} tr(A G_mm' A G_m'm)
//   ||R||^2 = (1/n^2) sum_{m,m'} |tr G_m'm|^2
// and eta follows from ||R - a b^T||^2 = ||R||^2 - 2 Re(a^H R conj(b)) +
// ||a||^2 ||b||^2.  The only q^2-sized work is writing the final time factor
// B-hat, a rank-np product (kernel lrk_emit_b).
//
// lrk_solve: one workgroup.  All eight waves accumulate the Gram matrix of the
// n p snapshot rows (FP64 sums of FP32 products) and the row sums that give
// the initialiser of Eq. (18), then run the iterations in FP64: the n^2 block
// products over all threads, EIG_{r_a} by cyclic Jacobi rotations on wave 0
// with the p x p matrix in registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kstap_internal.h"
#include "kstap_small_eig.h"

namespace kstap {
namespace {

using namespace small;

constexpr int kLrkMaxRows = 64;   // n * p
constexpr int kLrkMaxP = 8;

constexpr int kSolveThreads = 512;
constexpr int kSolveWaves = kSolveThreads / 64;
constexpr int kStageMax = 8192;             // staged samples per chunk (n p rows x chunk length)
constexpr int kPre = kStageMax / kSolveThreads;                 // staged samples per thread
constexpr int kMaxEnt = (kLrkMaxRows * (kLrkMaxRows + 1) / 2 + kLrkMaxRows + kSolveThreads - 1) / kSolveThreads;
// LDS region shared by the phases: the staged chunk (Gram), then the pair
// products T and the partial sums of M and tb (iterations).
constexpr size_t kOffT = 0;
constexpr size_t kOffPm = sizeof(dc) * kLrkMaxRows * kLrkMaxRows;    // after T (n^2 p^2 <= 64^2 entries)
constexpr size_t kOffPt = kOffPm + sizeof(dc) * kSolveThreads;
constexpr size_t kRegion = kOffPt + sizeof(double) * kSolveThreads;
static_assert(sizeof(float2) * (kStageMax + kLrkMaxRows) <= kRegion, "staged chunk fits the shared region");

// P: channels, a compile-time constant so that the p x p matrices of the
// iteration live in registers.
//
// Gram phase: entry e of the upper triangle (or row sum) of the n p snapshot
// rows belongs to one thread per sample group; every thread keeps its FP64
// sums of FP32 products in registers over all chunks (the chunks, as long as
// the LDS region allows for n p rows, are staged through LDS with the next
// one's global loads in flight while the current one is consumed) and the
// groups are added once at the end.
//
// Iterations: all threads form the n^2 products T_(m,m') = G_m'm A, then the
// partial sums of M = sum T_(m,m') G_mm' and tb = Re sum tr(T_(m,m') T_(m',m))
// over pair subsets; wave 0 adds them, takes EIG_{r_a} (parallel Jacobi, one
// lane per matrix entry) and the stop decision.
template <int P>
__global__ __launch_bounds__(kSolveThreads) void lrk_solve(const float2* __restrict__ X, LrkParams prm) {
  constexpr int p = P;
  const int n = prm.n, q = prm.q, np = n * p;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __shared__ dc sG[kLrkMaxRows * kLrkMaxRows];   // Gram of the snapshot rows
  __shared__ dc sRow[kLrkMaxRows];               // row sums
  __shared__ dc sA[kLrkMaxP * kLrkMaxP], sAp[kLrkMaxP * kLrkMaxP];
  __shared__ dc sH[kLrkMaxP * kLrkMaxP], sV[kLrkMaxP * kLrkMaxP], sM[kLrkMaxP * kLrkMaxP];
  __shared__ double sLam[kLrkMaxP];
  __shared__ int sStop;
  __shared__ __align__(16) char sReg[kRegion];
  float2* const sX = reinterpret_cast<float2*>(sReg);
  dc* const sT = reinterpret_cast<dc*>(sReg + kOffT);
  dc* const sPm = reinterpret_cast<dc*>(sReg + kOffPm);
  double* const sPt = reinterpret_cast<double*>(sReg + kOffPt);

  // ---- Gram matrix (upper triangle) and row sums
  const int ntri = np * (np + 1) / 2, nent = ntri + np;
  const bool grouped = nent <= kSolveThreads;
  const int G = grouped ? kSolveThreads / nent : 1;   // sample groups
  const int grp = grouped ? tid / nent : 0;
  int eu[kMaxEnt], ev[kMaxEnt];   // row u, column v of each entry (v < 0: row sum of u)
  int ne = 0;
#pragma unroll
  for (int j = 0; j < kMaxEnt; ++j) {
    const int e = grouped ? (j == 0 && grp < G ? tid - grp * nent : nent) : tid + j * kSolveThreads;
    eu[j] = 0;
    ev[j] = -1;
    if (e < nent) {
      ne = j + 1;
      if (e >= ntri) {
        eu[j] = e - ntri;
      } else {   // e -> (u, v), u <= v, row-major over the upper triangle
        int u = 0, rem = e;
        while (rem >= np - u) {
          rem -= np - u;
          ++u;
        }
        eu[j] = u;
        ev[j] = u + rem;
      }
    }
  }
  double ar[kMaxEnt], ai[kMaxEnt];
#pragma unroll
  for (int j = 0; j < kMaxEnt; ++j) ar[j] = ai[j] = 0.0;

  // chunk length: a power of two from 128 to 1024 with n p x chunk <= kStageMax
  int lch = 7;
  while (lch < 10 && (np << (lch + 1)) <= kStageMax) ++lch;
  const int chunk = 1 << lch, pitch = chunk + 1;   // padded LDS row (float2)
  float2 pre[kPre];   // element tid + 512 j of the chunk: row e >> lch, sample e & (chunk - 1)
  auto load_chunk = [&](int k0) {
    const int len = min(chunk, q - k0);
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int e = tid + j * kSolveThreads, u = e >> lch, k = e & (chunk - 1);
      pre[j] = (u < np && k < len) ? X[int64_t(u) * q + k0 + k] : make_float2(0.f, 0.f);
    }
  };
  const int nch = (q + chunk - 1) / chunk;
  load_chunk(0);
  for (int ch = 0; ch < nch; ++ch) {
    const int len = min(chunk, q - ch * chunk);
    __syncthreads();   // the previous chunk is consumed
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int e = tid + j * kSolveThreads, u = e >> lch, k = e & (chunk - 1);
      if (u < np) sX[u * pitch + k] = pre[j];
    }
    __syncthreads();
    if (ch + 1 < nch) load_chunk((ch + 1) * chunk);
    if (grouped) {
      // one entry per thread: four independent sums in flight
      if (ne > 0) {
        const float2* const ra = sX + eu[0] * pitch;
        const bool rowsum = ev[0] < 0;
        const float2* const rb = sX + (rowsum ? eu[0] : ev[0]) * pitch;
        double xr[4] = {0, 0, 0, 0}, xi[4] = {0, 0, 0, 0};
        int k = grp;
        for (; k + 3 * G < len; k += 4 * G) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float2 a = ra[k + t * G];
            const float2 b = rowsum ? make_float2(1.f, 0.f) : rb[k + t * G];   // a * conj(b)
            xr[t] += double(a.x) * double(b.x) + double(a.y) * double(b.y);
            xi[t] += double(a.y) * double(b.x) - double(a.x) * double(b.y);
          }
        }
        for (; k < len; k += G) {
          const float2 a = ra[k];
          const float2 b = rowsum ? make_float2(1.f, 0.f) : rb[k];
          xr[0] += double(a.x) * double(b.x) + double(a.y) * double(b.y);
          xi[0] += double(a.y) * double(b.x) - double(a.x) * double(b.y);
        }
        ar[0] += (xr[0] + xr[1]) + (xr[2] + xr[3]);
        ai[0] += (xi[0] + xi[1]) + (xi[2] + xi[3]);
      }
    } else {
      for (int k = 0; k < len; ++k) {
#pragma unroll
        for (int j = 0; j < kMaxEnt; ++j) {
          if (j < ne) {
            const float2 a = sX[eu[j] * pitch + k];
            const float2 b = ev[j] >= 0 ? sX[ev[j] * pitch + k] : make_float2(1.f, 0.f);   // a * conj(b)
            ar[j] += double(a.x) * double(b.x) + double(a.y) * double(b.y);
            ai[j] += double(a.y) * double(b.x) - double(a.x) * double(b.y);
          }
        }
      }
    }
  }
  __syncthreads();   // the staged chunk is dead: its region takes the group partials
  auto put = [&](int u, int v, dc s) {
    if (v < 0) {
      sRow[u] = s;
    } else {
      sG[u * np + v] = s;
      if (v != u) sG[v * np + u] = cj(s);
    }
  };
  if (grouped) {
    if (ne > 0) sPm[tid] = mk(ar[0], ai[0]);
    __syncthreads();
    if (tid < nent) {
      dc s = mk(0, 0);
      for (int g2 = 0; g2 < G; ++g2) s = add(s, sPm[g2 * nent + tid]);
      put(eu[0], ev[0], s);
    }
  } else {
#pragma unroll
    for (int j = 0; j < kMaxEnt; ++j)
      if (j < ne) put(eu[j], ev[j], mk(ar[j], ai[j]));
  }
  __syncthreads();

  auto G_ = [&](int m, int mm, int i, int j) -> dc { return sG[(m * p + i) * np + mm * p + j]; };
  const int npair = n * n;
  double normR2 = 0;
  if (wave == 0) {
    // ||R||^2 = ||S||^2 = (1/n^2) sum_{m,m'} |tr G_m'm|^2
    double nr = 0;
    for (int t = lane; t < npair; t += 64) {
      const int m = t / n, mm = t - (t / n) * n;
      dc tr = mk(0, 0);
      for (int i = 0; i < p; ++i) tr = add(tr, G_(mm, m, i, i));
      nr += ab2(tr);
    }
    normR2 = wave_sum(nr) / (double(n) * n);
    // initialiser (Eq. (18)): A0 = (1/(n q^2)) sum_m s_m s_m^H, s_m the row
    // sums; fallback R vec(I_q) = (1/n) sum_m G_mm when ||A0|| is negligible.
    // Lane e < p^2 holds entry (e / p, e % p).
    double an = 0;
    if (lane < p * p) {
      const int i = lane / p, j = lane - (lane / p) * p;
      dc s = mk(0, 0);
      for (int m = 0; m < n; ++m) s = add(s, mul(sRow[m * p + i], cj(sRow[m * p + j])));
      sA[lane] = scl(s, 1.0 / (double(n) * q * q));
      an = ab2(sA[lane]);
    }
    an = wave_sum(an);
    if (an <= 1e-24 * normR2 && lane < p * p) {
      const int i = lane / p, j = lane - (lane / p) * p;
      dc s = mk(0, 0);
      for (int m = 0; m < n; ++m) s = add(s, G_(m, m, i, j));
      sA[lane] = scl(s, 1.0 / n);
    }
    if (lane == 0) sStop = !(normR2 > 0.0);
  }
  __syncthreads();
  const bool zero = sStop != 0;

  double eta = 0, eta_prev = INFINITY, bn2 = 0;
  int iters = 0;
  constexpr int PP = P * P;
  constexpr int kSplit = kSolveThreads / PP;   // pair subsets of the partial sums
  while (!zero) {
    // T_(m,m') = G_m'm A, pair t = m n + m'
    for (int task = tid; task < npair * PP; task += kSolveThreads) {
      const int t = task / PP, ik = task - t * PP, i = ik / P, k = ik - i * P;
      const int m = t / n, mm = t - m * n;
      dc s = mk(0, 0);
#pragma unroll
      for (int l = 0; l < P; ++l) s = add(s, mul(G_(mm, m, i, l), sA[l * P + k]));
      sT[task] = s;
    }
    __syncthreads();
    // partial sums of M[i][j] = sum_t (T_t G_mm')[i][j] and of
    // tb = Re sum_t tr(T_(m,m') T_(m',m)) (this thread's term: entry (i, j))
    {
      dc pm = mk(0, 0);
      double pt = 0;
      const int o = tid % PP, s = tid / PP;
      if (s < kSplit) {
        const int i = o / P, j = o - (o / P) * P;
        for (int t = s; t < npair; t += kSplit) {
          const int m = t / n, mm = t - m * n;
#pragma unroll
          for (int k = 0; k < P; ++k) pm = add(pm, mul(sT[t * PP + i * P + k], G_(m, mm, k, j)));
          pt += mul(sT[t * PP + i * P + j], sT[(mm * n + m) * PP + j * P + i]).x;
        }
      }
      sPm[tid] = pm;
      sPt[tid] = pt;
    }
    __syncthreads();
    if (wave == 0) {
      double an2 = 0;
      for (int e = 0; e < PP; ++e) an2 += ab2(sA[e]);
      const double c = 1.0 / (double(n) * an2);
      double tb = 0;
      for (int j = lane; j < kSolveThreads; j += 64) tb += sPt[j];
      tb = wave_sum(tb);
      if (lane < PP) {
        dc s = mk(0, 0);
        for (int g2 = 0; g2 < kSplit; ++g2) s = add(s, sPm[g2 * PP + lane]);
        sM[lane] = s;
      }
      lane_sync();
      bn2 = c * c * tb;                           // ||b||^2
      const double sa = c / (double(n) * bn2);    // A' = R conj(b) / ||b||^2 = sa M
      // EIG_{r_a} of the Hermitian part of A'
      if (lane < PP) {
        const int i = lane / p, j = lane - (lane / p) * p;
        sAp[lane] = scl(sM[lane], sa);
        sH[lane] = scl(add(scl(sM[i * p + j], sa), cj(scl(sM[j * p + i], sa))), 0.5);
      }
      lane_sync();
      {
        constexpr int PE = (P + 1) / 2 * 2;
        const int r = lane / PE, cc = lane - (lane / PE) * PE;
        const bool real = r < P && cc < P;   // not the pad row or column, nor past PE^2
        dc h = real ? sH[r * P + cc] : mk(0, 0), v;
        jacobi_par<P>(h, v, lane);
        if (real) {
          sV[r * P + cc] = v;
          if (r == cc) sLam[r] = h.x;
        }
      }
      lane_sync();
      // the r_a largest algebraic eigenvalues (uniform selection on every lane)
      dc anew = mk(0, 0);
      {
        unsigned used = 0;
        const int i = lane / p, j = lane - (lane / p) * p;
        for (int r = 0; r < prm.r_a; ++r) {
          int best = -1;
          for (int k = 0; k < p; ++k)
            if (!((used >> k) & 1u) && (best < 0 || sLam[k] > sLam[best])) best = k;
          used |= 1u << best;
          if (lane < PP) anew = add(anew, scl(mul(sV[i * p + best], cj(sV[j * p + best])), sLam[best]));
        }
      }
      lane_sync();
      double na = 0, cross = 0;
      if (lane < PP) {
        sA[lane] = anew;
        na = ab2(anew);
        cross = mul(cj(anew), sAp[lane]).x;
      }
      na = wave_sum(na);
      cross = wave_sum(cross);
      ++iters;
      // eta^2 = (||R||^2 - 2 ||b||^2 Re<A, A'> + ||A||^2 ||b||^2) / ||R||^2
      const double r2 = normR2 - 2.0 * bn2 * cross + na * bn2;
      const double e = sqrt(fmax(r2, 0.0) / normR2);
      eta = e;
      const bool stop =
          iters >= prm.max_iter || (prm.eps > 0.0 && iters >= prm.min_iter && fabs(e - eta_prev) <= prm.eps);
      eta_prev = e;
      if (lane == 0) sStop = stop ? 1 : 0;
    }
    __syncthreads();
    if (sStop) break;
  }
  if (wave != 0) return;
  if (lane < PP) prm.A[lane] = zero ? make_float2(0.f, 0.f) : make_float2(float(sA[lane].x), float(sA[lane].y));
  if (lane == 0 && prm.stats) {
    prm.stats[0] = zero ? 0.0 : eta;
    prm.stats[1] = double(iters);
    prm.stats[2] = sqrt(normR2);
    prm.stats[3] = zero ? 0.0 : sqrt(bn2);
  }
}

// Final time factor B-hat[k][l] = c sum_{m, j} W_m[k][j] conj(X_m[j][l]) with
// W_m = X_m^T conj(A) (q x p) and c = 1 / (n ||A||^2): a rank-np product,
// bound by writing q^2 complex values.  64 x 64 outputs per 256-thread block,
// each thread 4 rows x 4 columns (columns strided by 16 so that each store
// instruction writes 16 consecutive entries per row).  The LDS operands are
// sized for the actual n p (dynamic shared memory), so that many blocks share
// a compute unit and keep enough stores in flight.
constexpr int kTile = 64;
__global__ __launch_bounds__(256) void lrk_emit_b(const float2* __restrict__ X, LrkParams prm) {
  const int n = prm.n, p = prm.p, q = prm.q, np = n * p;
  extern __shared__ float2 dyn[];
  float2* const sW = dyn;                        // [kTile][np + 1]: W for the tile's rows k
  float2* const sXc = dyn + kTile * (np + 1);    // [np][kTile + 1]: conj(X) for the tile's columns l
  __shared__ float2 sAc[kLrkMaxP * kLrkMaxP];
  __shared__ float sC;
  const int tid = threadIdx.x;
  const int k0 = blockIdx.y * kTile, l0 = blockIdx.x * kTile;
  if (tid < p * p) sAc[tid] = make_float2(prm.A[tid].x, -prm.A[tid].y);   // conj(A)
  if (tid == 0) {
    float an = 0.f;
    for (int e = 0; e < p * p; ++e) an += prm.A[e].x * prm.A[e].x + prm.A[e].y * prm.A[e].y;
    sC = an > 0.f ? 1.f / (float(n) * an) : 0.f;
  }
  // conj(X) rows for the tile's columns (coalesced over l)
  for (int e = tid; e < np * kTile; e += 256) {
    const int u = e / kTile, ll = e - (e / kTile) * kTile;
    const int l = l0 + ll;
    const float2 x = (l < q) ? X[int64_t(u) * q + l] : make_float2(0.f, 0.f);
    sXc[u * (kTile + 1) + ll] = make_float2(x.x, -x.y);
  }
  __syncthreads();
  // W[k][(m, j)] = sum_i X_m[i][k] conj(A)[i][j], consecutive threads over k
  for (int e = tid; e < kTile * np; e += 256) {
    const int u = e / kTile, kk = e - (e / kTile) * kTile;
    const int m = u / p, j = u - (u / p) * p;
    const int k = k0 + kk;
    float2 sum = make_float2(0.f, 0.f);
    if (k < q) {
      for (int i = 0; i < p; ++i) {
        const float2 x = X[(int64_t(m) * p + i) * q + k];
        const float2 a = sAc[i * p + j];
        sum.x += x.x * a.x - x.y * a.y;
        sum.y += x.x * a.y + x.y * a.x;
      }
    }
    sW[kk * (np + 1) + u] = sum;
  }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;   // columns tx + 16 c, rows ty + 16 r
  float2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = make_float2(0.f, 0.f);
  for (int u = 0; u < np; ++u) {
    float2 w[4], x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = sW[(ty + 16 * r) * (np + 1) + u];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = sXc[u * (kTile + 1) + tx + 16 * c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[r][c].x = fmaf(w[r].x, x[c].x, fmaf(-w[r].y, x[c].y, acc[r][c].x));
        acc[r][c].y = fmaf(w[r].x, x[c].y, fmaf(w[r].y, x[c].x, acc[r][c].y));
      }
  }
  const float cs = sC;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = k0 + ty + 16 * r;
    if (k >= q) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int l = l0 + tx + 16 * c;
      if (l < q) prm.B[int64_t(k) * q + l] = make_float2(acc[r][c].x * cs, acc[r][c].y * cs);
    }
  }
}

}  // namespace

int launch_lrkron(const float2* X, const LrkParams& prm, hipStream_t stream) {
  if (prm.n * prm.p > kLrkMaxRows || prm.p > kLrkMaxP || prm.p < 1 || prm.q < 1) return hipErrorInvalidValue;
  switch (prm.p) {
    case 1: hipLaunchKernelGGL(lrk_solve<1>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 2: hipLaunchKernelGGL(lrk_solve<2>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 3: hipLaunchKernelGGL(lrk_solve<3>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 4: hipLaunchKernelGGL(lrk_solve<4>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 5: hipLaunchKernelGGL(lrk_solve<5>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 6: hipLaunchKernelGGL(lrk_solve<6>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 7: hipLaunchKernelGGL(lrk_solve<7>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    default: hipLaunchKernelGGL(lrk_solve<8>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !prm.B) return e;
  const unsigned t = unsigned((prm.q + kTile - 1) / kTile);
  const int np = prm.n * prm.p;
  const size_t lds = sizeof(float2) * (size_t(kTile) * (np + 1) + size_t(np) * (kTile + 1));
  hipLaunchKernelGGL(lrk_emit_b, dim3(t, t), dim3(256), lds, stream, X, prm);
  return hipGetLastError();
}

}  // namespace kstap
