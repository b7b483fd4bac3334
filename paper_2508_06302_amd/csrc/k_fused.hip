// Fused trajectory kernel: state integration and sensitivity propagation of one
// trajectory in one work-group (App. E), for half bandwidths up to 16.
//
// Work-group (p, w): trajectory w, sensitivity columns [p*64*NCW, (p+1)*64*NCW).
// A four-stage pipeline, one barrier per stage step:
//   wave 0  state      step k: q_k -> q_{k+1} (Eqs. E4-E7).  Eq. (E6) is solved by a
//                      chord Newton whose matrix is the exact tangent at a two-step
//                      prediction of q_{k+1}, factored one step ahead by wave 1; if the
//                      contraction is poor the wave refactors T at its own iterate.
//   wave 1  chord      step k: T(q^_{k+2}) with q^_{k+2} = q_k + 2h u_k,
//                      assembled and factored (banded LDL^T) for state step k + 1.
//   wave 2  tangent    step k: T(q_k) = S + K_t(q_k) at the converged state, factored.
//   waves 3.. columns  step k: advance [Q; U; A] from step k-2 to k-1 with the factor
//                      of T(q_{k-1}) (exact derivative of the converged discrete map,
//                      Eqs. E8-E9); in step 0 they form Q_0, U_0, A_0.
// The chord stops once ||dq||_inf <= 1e-3 tol ||q||_inf, or once the linear-convergence
// bound rho/(1-rho) ||dq|| on the remaining error (rho the observed contraction) is below
// 1e-2 tol ||q||: the flow amplifies per-step errors over a period, so the chord must
// leave no more error than a full Newton step that stops at tol.  An update that stops
// shrinking below tol ||q|| is the FP64 noise floor of the residual and ends the step.
// On poor contraction (rho >= 1/4) above tol the state wave refactors T at the current
// iterate once and continues (stagnation below 1e3 tol with that fresh tangent is the
// noise floor); if that fails too, or the chord spends maxit iterations, it restarts
// from the predictor with full Newton and a fresh budget of maxit iterations, which
// stops on ||dq||_inf <= tol ||q||_inf or stagnation below 1e3 tol.
//
// Banded data are padded to the compile-time half bandwidth BW >= bw with zeros:
//   full rows  [n][2BW+1]   entry (i, j) at [i][j - i + BW]      (global, per point)
//   LDL^T      [n+BW][BW+1] entry (j + r, j) at [BW + j][r]; [BW + j][0] = 1 / d_j;
//                           the BW leading columns are zero so sweeps need no guards.
#include <climits>
#include <type_traits>
#include <cmath>

#include "band_ldlt.h"
#include "fse_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct FusedArgs {
  TrajParams P;
  const double *Kb0;                       // unpadded full rows [n][2bw+1]
  const double *F;                         // loads [e][n]
  const int32_t *f2_ptr, *f2_jk;
  const double *f2_v;
  const int32_t *f3_ptr, *f3_jkl;
  const double *f3_v;
  const uint32_t *f2_pk, *f3_pk;           // packed indices (see fse_ctx)
  int nnz2, nnz3;
  const double *omega;                     // [B][d]
  const int32_t *sidx, *Sdim;
  const double *q0, *u0;                   // [n][ldw]
  int ldw;
  double *zT;                              // [2n][ldw]
  double *qhist;                           // [S1+1][n][ldw] rows 1..S1 written, or null
  double *Phi;                             // [W][2n][2n] or null
  void *colQ, *colU, *colA, *colY;         // column state [n][2n] blocks (CT elements)
  size_t colQ_ws, colU_ws, colA_ws, colY_ws;  // element stride between trajectories
  DevStatus *st;
};

// Per-point padded bands: S = w1^2 c0 M + w1 c2 D + K, w1^2 M, w1 D; and K itself.
template <int BW>
__global__ void k_point_bands(TrajParams P, const double *__restrict__ Mb, const double *__restrict__ Db,
                              const double *__restrict__ Kb, const double *__restrict__ omega, int B,
                              double *__restrict__ Sp, double *__restrict__ Mwp, double *__restrict__ Dwp,
                              double *__restrict__ Kp) {
  constexpr int W2 = 2 * BW + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = B * P.n * W2;
  if (idx >= total) return;
  const int t = idx % W2;
  const int i = (idx / W2) % P.n;
  const int b = idx / (W2 * P.n);
  const double w1 = omega[b * P.d];
  const int j = i - BW + t;
  const int tb = j - i + P.bw;
  double m = 0.0, dd = 0.0, k = 0.0;
  if (j >= 0 && j < P.n && tb >= 0 && tb <= 2 * P.bw) {
    const size_t e = (size_t)i * (2 * P.bw + 1) + tb;
    m = Mb[e];
    dd = Db[e];
    k = Kb[e];
  }
  Mwp[idx] = w1 * w1 * m;
  Dwp[idx] = w1 * dd;
  Sp[idx] = w1 * w1 * P.c0 * m + w1 * P.c2 * dd + k;
  if (b == 0) Kp[idx] = k;
}

__device__ inline double forcing_cos(const FusedArgs &a, int f, double phi1, const double *om, int s,
                                    double phi0) {
  if (f == 0) return cos(phi0 + phi1);
  const double ph = kTwoPi * (double)a.sidx[(f - 1) * a.P.St + s] / (double)a.Sdim[f - 1];
  return cos(ph + om[f] / om[0] * phi1);
}

// rows per block in the sensitivity sweeps: every block is one round trip of loads, so
// larger blocks keep more bytes in flight; 16 where the registers allow it
template <int BW> constexpr int rows_per_block() { return BW == 6 ? 16 : 8; }
// Chord stop: an update below kChordFloor tol |q| ends the step; otherwise the linear
// error bound must fall below kChordBound tol |q|.
constexpr double kChordFloor = 1e-3;
constexpr double kChordBound = 1e-2;

// One sensitivity step for the column owned by this lane (Eqs. E8-E9).  Column state
// [Q; U; A] and the solve scratch Y are stored as CT (double, or float for the mixed
// path); arithmetic is FP64.  Pass A walks the rows upwards in blocks of kRB: the block's
// rows of Q, U, A are loaded together (the 2 BW rows of overlap stay in registers), the
// right-hand side w1^2 M (c0 Q + c1 U + c3 A) + w1 D (c2 Q + d1 U + d2 A) is formed and immediately
// forward-substituted with the unit lower factor.  Pass B walks back down: D^-1 and the
// backward substitution, then the Newmark update of [Q; U; A].
template <int BW, typename CT>
__device__ void sens_step(const double *F_, const double *__restrict__ Mwp_, const double *__restrict__ Dwp_,
                          int n, int n2, double c0, double c1, double c2, double c3, double d1, double d2,
                          CT *__restrict__ Qc_,
                          CT *__restrict__ Uc_, CT *__restrict__ Ac_, CT *__restrict__ Yc_) {
  // The factor lives in LDS and the column state and bands in global memory; typed pointers
  // keep every access an LDS or a global instruction where the call is not inlined.
  typedef __attribute__((address_space(1))) CT gCT;
  typedef __attribute__((address_space(1))) const double gcdouble;
  const lds_double *F = (const lds_double *)F_;
  gcdouble *Mwp = (gcdouble *)Mwp_, *Dwp = (gcdouble *)Dwp_;
  gCT *Qc = (gCT *)Qc_, *Uc = (gCT *)Uc_, *Ac = (gCT *)Ac_, *Yc = (gCT *)Yc_;
  constexpr int bp = BW + 1, W2 = 2 * BW + 1;
  constexpr int kRB = rows_per_block<BW>();
  constexpr int NR = kRB + 2 * BW;
  double v1[NR], v2[NR], yw[BW];
#pragma unroll
  for (int t = 0; t < BW; ++t) yw[t] = 0.0;
  // rows -BW .. BW-1 of the first window (rows 0 .. BW-1 loaded together)
  {
    CT Qn[BW], Un[BW], An[BW];
#pragma unroll
    for (int t = 0; t < BW; ++t) {
      const int j = min(t, n - 1);
      Qn[t] = Qc[(size_t)j * n2];
      Un[t] = Uc[(size_t)j * n2];
      An[t] = Ac[(size_t)j * n2];
    }
#pragma unroll
    for (int t = 0; t < BW; ++t) {
      v1[t] = 0.0;
      v2[t] = 0.0;
      const bool in = t < n;
      const double Qj = in ? (double)Qn[t] : 0.0, Uj = in ? (double)Un[t] : 0.0;
      const double Aj = in ? (double)An[t] : 0.0;
      v1[BW + t] = c0 * Qj + c1 * Uj + c3 * Aj;
      v2[BW + t] = c2 * Qj + d1 * Uj + d2 * Aj;
    }
  }
  for (int i0 = 0; i0 < n; i0 += kRB) {
    // new rows i0+BW .. i0+BW+kRB-1 into window slots 2BW .. NR-1; every load is issued
    // (rows past n read row n-1 and are zeroed afterwards) before any is used
    CT Qn[kRB], Un[kRB], An[kRB];
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      const int j = min(i0 + BW + d, n - 1);
      Qn[d] = Qc[(size_t)j * n2];
      Un[d] = Uc[(size_t)j * n2];
      An[d] = Ac[(size_t)j * n2];
    }
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      const bool in = i0 + BW + d < n;
      const double Qj = in ? (double)Qn[d] : 0.0, Uj = in ? (double)Un[d] : 0.0;
      const double Aj = in ? (double)An[d] : 0.0;
      v1[2 * BW + d] = c0 * Qj + c1 * Uj + c3 * Aj;
      v2[2 * BW + d] = c2 * Qj + d1 * Uj + d2 * Aj;
    }
    double yb[kRB];
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      const int i = i0 + d;
      double acc = 0.0;
      if (i < n) {
        gcdouble *mr = Mwp + (size_t)i * W2;
        gcdouble *dr = Dwp + (size_t)i * W2;
#pragma unroll
        for (int t = 0; t < W2; ++t) acc += mr[t] * v1[d + t] + dr[t] * v2[d + t];
#pragma unroll
        for (int t = BW; t >= 1; --t) acc -= F[(i - t) * bp + t] * yw[t - 1];
      }
#pragma unroll
      for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
      yw[0] = acc;
      yb[d] = acc;
    }
#pragma unroll
    for (int d = 0; d < kRB; ++d)
      if (i0 + d < n) Yc[(size_t)(i0 + d) * n2] = (CT)yb[d];
    // slide the window by kRB rows
#pragma unroll
    for (int t = 0; t < 2 * BW; ++t) {
      v1[t] = v1[t + kRB];
      v2[t] = v2[t + kRB];
    }
  }
  // pass B: backward substitution and the Newmark update of [Q; U; A]
#pragma unroll
  for (int t = 0; t < BW; ++t) yw[t] = 0.0;
  const int nb = (n + kRB - 1) / kRB;
  for (int blk = nb - 1; blk >= 0; --blk) {
    const int i0 = blk * kRB;
    CT ry[kRB], rq[kRB], ru[kRB], ra[kRB];
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      const int i = min(i0 + d, n - 1);
      ry[d] = Yc[(size_t)i * n2];
      rq[d] = Qc[(size_t)i * n2];
      ru[d] = Uc[(size_t)i * n2];
      ra[d] = Ac[(size_t)i * n2];
    }
    double yb[kRB], qb[kRB], ub[kRB], ab[kRB];
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      yb[d] = (double)ry[d];
      qb[d] = (double)rq[d];
      ub[d] = (double)ru[d];
      ab[d] = (double)ra[d];
    }
#pragma unroll
    for (int d = kRB - 1; d >= 0; --d) {
      const int i = i0 + d;
      if (i >= n) continue;
      double x = yb[d] * F[i * bp];
#pragma unroll
      for (int t = BW; t >= 1; --t) x -= F[i * bp + t] * yw[t - 1];
#pragma unroll
      for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
      yw[0] = x;
      yb[d] = x;
    }
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      const int i = i0 + d;
      if (i >= n) continue;
      const double dQ = yb[d] - qb[d];
      Uc[(size_t)i * n2] = (CT)(c2 * dQ - d1 * ub[d] - d2 * ab[d]);
      Ac[(size_t)i * n2] = (CT)(c0 * dQ - c1 * ub[d] - c3 * ab[d]);
      Qc[(size_t)i * n2] = (CT)yb[d];
    }
  }
}

template <int BW, typename CT>
__global__ __launch_bounds__(320) void k_fused(FusedArgs a, const double *__restrict__ Sp_all,
                                               const double *__restrict__ Mwp_all,
                                               const double *__restrict__ Dwp_all,
                                               const double *__restrict__ Kp) {
  constexpr int bp = BW + 1, W2 = 2 * BW + 1;
  // the chord factor is kept in FP32 for half bandwidths up to 6 (one-lane FP32 solve)
  constexpr bool kChord32 = BW <= 6;
  extern __shared__ __attribute__((aligned(16))) double smem[];
  const TrajParams &P = a.P;
  const int n = P.n, n2 = 2 * n;
  const int w = blockIdx.y;
  const int b = w / P.St, s = w - b * P.St;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ncw = (blockDim.x >> 6) - 3;
  const double *om = a.omega + b * P.d;
  // read-only per-point bands; __restrict__ lets uniform row reads use the scalar path
  const double *__restrict__ Sp = Sp_all + (size_t)b * n * W2;
  const double *__restrict__ Mwp = Mwp_all + (size_t)b * n * W2;
  const double *__restrict__ Dwp = Dwp_all + (size_t)b * n * W2;

  const size_t fb = (size_t)(n + BW) * bp;   // one padded factor buffer
  const int n1 = n + 1;                      // state vector stride
  double *FM = smem;                         // factor of w1^2 M
  double *KtB = FM + fb;                     // lower band of K + K_t(q0) (same padding)
  // FM and KtB serve the prologue and step 0 only; from step 1 on they hold an LDS copy of
  // the per-point band S [n][2BW+1] (n (2BW+1) <= 2 fb), read by every residual and assembly
  double *Sl = FM;
  const lds_double *SlL = (const lds_double *)Sl;
  double *FT0 = KtB + fb;                    // factors of T(q_k), double buffered
  double *FT1 = FT0 + fb;
  double *CB0 = FT1 + fb;                    // chord factor T(predicted q): FP64 work buffer,
  double *CB1 = kChord32 ? CB0 : CB0 + fb;   // double buffered unless the chord is FP32
  double *FR = CB1 + fb;                     // state-wave refresh factor
  double *q = FR + fb;
  double *u = q + n1;
  double *acc = u + n1;
  double *qn = acc + n1;
  double *bv = qn + n1;
  double *r = bv + n1;
  double *qs0 = r + n1;                      // q_k handed to the factor wave
  double *qs1 = qs0 + n1;
  double *pq0 = qs1 + n1;                    // two-step predictions handed to the chord wave
  double *pq1 = pq0 + n1;
  double *cs = pq1 + n1;                     // forcing cosines [8]
  double *tv2 = cs + 8;                      // staged polynomial forces
  double *tv3 = tv2 + a.nnz2;
  int *tp2 = reinterpret_cast<int *>(tv3 + a.nnz3);
  int *tp3 = tp2 + (n + 1);
  uint32_t *ti2 = reinterpret_cast<uint32_t *>(tp3 + (n + 1));
  uint32_t *ti3 = ti2 + a.nnz2;
  // FP32 chord factors (double buffered) and right-hand side, 16-byte aligned
  const int crows = chord_rows(n);
  char *const lds0 = reinterpret_cast<char *>(smem);
  const size_t cfo = ((size_t)(reinterpret_cast<char *>(ti3 + 2 * a.nnz3) - lds0) + 15) & ~(size_t)15;
  float *CF0 = reinterpret_cast<float *>(lds0 + cfo);
  float *CF1 = CF0 + 8 * crows;
  float *RF = CF1 + 8 * crows;
  const TensLds tl{(const lds_int *)tp2, (const lds_int *)tp3, (const lds_u32 *)ti2, (const lds_u32 *)ti3,
                   (const lds_double *)tv2, (const lds_double *)tv3};
  // the FP32 chord buffers need 16-byte alignment (b128 accesses); without it the chord
  // iterations use the FP64 factor
  const bool chord32 = kChord32 && (reinterpret_cast<uintptr_t>(CF0) & 15) == 0;
  __shared__ int s_fail_step;
  __shared__ int s_flags;
  // phase of forcing 1 at the start (multiple-shooting segments), read from LDS once per step
  // so that no register carries it across the step loop
  __shared__ double s_phi0;

  // ============================================================ prologue
  for (int e = threadIdx.x; e < (int)(FR + fb - smem); e += blockDim.x) smem[e] = 0.0;
  if constexpr (kChord32)
    for (int e = threadIdx.x; e < 17 * crows; e += blockDim.x) CF0[e] = 0.0f;
  for (int e = threadIdx.x; e <= n; e += blockDim.x) {
    tp2[e] = a.f2_ptr[e];
    tp3[e] = a.f3_ptr[e];
  }
  for (int e = threadIdx.x; e < a.nnz2; e += blockDim.x) {
    tv2[e] = a.f2_v[e];
    ti2[e] = a.f2_pk[e];
  }
  for (int e = threadIdx.x; e < a.nnz3; e += blockDim.x) {
    tv3[e] = a.f3_v[e];
    ti3[2 * e] = a.f3_pk[2 * e];
    ti3[2 * e + 1] = a.f3_pk[2 * e + 1];
  }
  if (threadIdx.x == 0) {
    s_fail_step = INT_MAX;
    s_flags = 0;
    s_phi0 = P.phib * b;
  }
  __syncthreads();
  if (wave == 0 || wave == 2) {
    for (int i = lane; i < n; i += 64) {
      const double qi = a.q0[(size_t)i * a.ldw + w];
      if (wave == 0) {
        q[i] = qi;
        u[i] = a.u0[(size_t)i * a.ldw + w];
      } else {
        qs0[i] = qi;
      }
    }
  }
  __syncthreads();
  if (wave == 2) {
    // w1^2 M, K + K_t(q0) and T(q0) = S + K_t(q0) lower bands; factor w1^2 M and T(q0)
    assemble_T<BW>(tl, n, Sp, qs0, FT0, lane);
    assemble_T<BW>(tl, n, Kp, qs0, KtB, lane);
    for (int pos = lane; pos < n * bp; pos += 64) {
      const int m = pos / bp, rr = pos - m * bp, i = m + rr;
      FM[BW * bp + pos] = i < n ? Mwp[(size_t)i * W2 + (BW - rr)] : 0.0;
    }
    wave_sync();
    if (lane == 0) {
      bool ok = ldlt_serial<BW>(FM, n);
      ok = ldlt_serial<BW>(FT0, n) && ok;
      if (!ok) s_flags |= DEV_SINGULAR;
    }
  }
  if (wave == 0) {
    if (lane < P.e) cs[lane] = forcing_cos(a, lane, 0.0, om, s, s_phi0);
    wave_sync();
    // a0 right-hand side: e0 - w1 D u0 - K q0 - f_nl(q0)
    for (int i = lane; i < n; i += 64) {
      double v = 0.0;
      for (int f = 0; f < P.e; ++f) v += a.F[(size_t)f * n + i] * cs[f];
#pragma unroll
      for (int t = 0; t < W2; ++t) {
        const int j = i - BW + t;
        if (j < 0 || j >= n) continue;
        const int tb = j - i + P.bw;
        const double k = (tb >= 0 && tb <= 2 * P.bw) ? a.Kb0[(size_t)i * (2 * P.bw + 1) + tb] : 0.0;
        v -= Dwp[(size_t)i * W2 + t] * u[j] + k * q[j];
      }
      acc[i] = v - fnl_row(tl, q, i);
    }
  }
  __syncthreads();
  if (wave == 0) {
    if (lane == 0) ldlt_solve_serial<BW>(FM, n, acc);
    wave_sync();
    // first-order predictions q^_1 = q0 + h u0 (chord of step 0, into qn) and
    // q^_2 = q0 + 2h u0 (chord of step 1, into pq0)
    for (int i = lane; i < n; i += 64) {
      qn[i] = q[i] + P.h * u[i];
      pq0[i] = q[i] + 2.0 * P.h * u[i];
    }
  }
  __syncthreads();
  if (wave == 1) {
    assemble_T<BW>(tl, n, Sp, qn, CB0, lane);
    wave_sync();
    if (lane == 0 && !ldlt_serial<BW>(CB0, n)) s_flags |= DEV_SINGULAR;
    if constexpr (kChord32) {
      wave_sync();
      chord_to_f32<BW>(CB0, n, CF0, lane);
    }
  }
  __syncthreads();

  // ============================================================ pipeline
  const int c = blockIdx.x * (64 * ncw) + (wave - 3) * 64 + lane;
  const bool colw = wave >= 3 && c < n2 && a.Phi != nullptr;
  CT *Qc = static_cast<CT *>(a.colQ) + (size_t)w * a.colQ_ws + c;
  CT *Uc = static_cast<CT *>(a.colU) + (size_t)w * a.colU_ws + c;
  CT *Ac = static_cast<CT *>(a.colA) + (size_t)w * a.colA_ws + c;
  CT *Yc = static_cast<CT *>(a.colY) + (size_t)w * a.colY_ws + c;
  int max_it = 0;
  unsigned long long tot_it = 0;
  const int last = a.Phi ? P.S1 + 1 : P.S1 - 1;

  for (int k = 0; k <= last; ++k) {
    if (wave == 0 && k < P.S1) {
      // ---------------- state step k: q_k -> q_{k+1}; chord matrix CB[k&1] = T(q^_{k+1})
      const double *Fc = (k & 1) ? CB1 : CB0;
      const float *Fc32 = (k & 1) ? CF1 : CF0;
      double *qsn = ((k + 1) & 1) ? qs1 : qs0;
      double *pqn = ((k + 1) & 1) ? pq1 : pq0;
      const double phi1 = (double)(k + 1) * P.h;
      const bool slds = k >= 1;  // the band copy is in place (this wave writes it in step 1)
      if (k == 1) {
        for (int e = lane; e < n * W2; e += 64) Sl[e] = Sp[e];
      }
      if (lane < P.e) cs[lane] = forcing_cos(a, lane, phi1, om, s, s_phi0);
      wave_sync();
      for (int i = lane; i < n; i += 64) {
        double v = 0.0;
        for (int f = 0; f < P.e; ++f) v += a.F[(size_t)f * n + i] * cs[f];
#pragma unroll
        for (int t = 0; t < W2; ++t) {
          const int j = i - BW + t;
          if (j < 0 || j >= n) continue;
          v += Mwp[(size_t)i * W2 + t] * (P.c0 * q[j] + P.c1 * u[j] + P.c3 * acc[j]) +
               Dwp[(size_t)i * W2 + t] * (P.c2 * q[j] + P.d1 * u[j] + P.d2 * acc[j]);
        }
        bv[i] = v;
        qn[i] = q[i] + P.h * u[i] + 0.5 * P.h * P.h * acc[i];
      }
      wave_sync();
      double prev = INFINITY;
      bool conv = false, full = false, refreshed = false;
      const double *Fcur = Fc;
      int it = 0, itc = 0;  // total iterations; iterations of the current mode (chord / full)
      while (!conv) {
        if (itc >= P.maxit) {
          if (full) break;
          // chord budget spent: restart from the predictor with full Newton
          for (int i = lane; i < n; i += 64) qn[i] = q[i] + P.h * u[i] + 0.5 * P.h * P.h * acc[i];
          wave_sync();
          full = true;
          prev = INFINITY;
          itc = 0;
        }
        ++it;
        ++itc;
        if (full) {
          // full Newton: exact tangent at the current iterate
          if (slds)
            assemble_T<BW, true>(tl, n, Sl, qn, FR, lane);
          else
            assemble_T<BW>(tl, n, Sp, qn, FR, lane);
          wave_sync();
          if (lane == 0 && !ldlt_serial<BW>(FR, n)) s_flags |= DEV_SINGULAR;
          wave_sync();
        }
        // the FP32 chord solve serves the chord iterations; full Newton and the refreshed
        // tangent use the FP64 factor
        const bool c32 = chord32 && !full && Fcur == Fc;
        for (int i = lane; i < n; i += 64) {
          double v = fnl_row(tl, qn, i) - bv[i];
#pragma unroll
          for (int t = 0; t < W2; ++t) {
            const int j = i - BW + t;
            if (j < 0 || j >= n) continue;
            const size_t e = (size_t)i * W2 + t;
            v += (slds ? SlL[e] : Sp[e]) * qn[j];
          }
          r[i] = v;
          if (c32) RF[i] = (float)v;
        }
        // padding rows of the FP32 right-hand side stay zero even after a non-finite residual
        if (c32)
          for (int i = n + lane; i < crows; i += 64) RF[i] = 0.0f;
        wave_sync();
        if (lane == 0) {
          bool done = false;
          if constexpr (kChord32) {
            if (c32) {
              chord_solve_f32<BW>(Fc32, n, RF);
              done = true;
            }
          }
          if (!done) ldlt_solve_serial<BW>(full ? FR : Fcur, n, r);
        }
        wave_sync();
        double nd = 0.0, nq = 0.0;
        for (int i = lane; i < n; i += 64) {
          const double dq = c32 ? (double)RF[i] : r[i];
          const double v = qn[i] - dq;
          qn[i] = v;
          nd = fmax(nd, fabs(dq));
          nq = fmax(nq, fabs(v));
        }
        nd = wave_max(nd);
        nq = wave_max(nq);
        wave_sync();
        const bool finite = (nd == nd) && (nq == nq) && nd < INFINITY;
        const double tolq = P.tol * nq;
        const double rho = prev < INFINITY ? nd / prev : 1.0;
        if (full) {
          // quadratic convergence: same rule as a full Newton step (App. E reading)
          if (!finite) break;
          if (nd <= tolq || (nd <= 1e3 * tolq && nd > 0.5 * prev)) conv = true;
          prev = nd;
        } else if (finite && nd <= kChordFloor * tolq) {
          conv = true;
        } else if (finite && prev < INFINITY && rho < 0.25) {
          // linear convergence: stop once the remaining error bound rho/(1-rho) |dq| is
          // two decades below tol; the flow amplifies per-step errors over a period
          if (rho / (1.0 - rho) * nd <= kChordBound * tolq) conv = true;
          prev = nd;
        } else if (finite && prev == INFINITY) {
          prev = nd;
        } else if (finite && nd <= tolq) {
          conv = true;  // no further contraction below tol: FP64 noise floor of the residual
        } else if (finite && refreshed && nd <= 1e3 * tolq && rho > 0.5) {
          conv = true;  // stagnation with a fresh tangent: the noise floor lies above tol
        } else if (finite && !refreshed) {
          // poor contraction: refresh the chord matrix at the current iterate and go on
          if (slds)
            assemble_T<BW, true>(tl, n, Sl, qn, FR, lane);
          else
            assemble_T<BW>(tl, n, Sp, qn, FR, lane);
          wave_sync();
          if (lane == 0 && !ldlt_serial<BW>(FR, n)) s_flags |= DEV_SINGULAR;
          wave_sync();
          Fcur = FR;
          refreshed = true;
          prev = INFINITY;
        } else {
          // poor contraction or divergence: restart from the predictor with full Newton
          for (int i = lane; i < n; i += 64) qn[i] = q[i] + P.h * u[i] + 0.5 * P.h * P.h * acc[i];
          wave_sync();
          full = true;
          prev = INFINITY;
          itc = 0;
        }
      }
      if (!conv && lane == 0) {
        s_flags |= DEV_NOCONV;
        if (k < s_fail_step) s_fail_step = k;
      }
      max_it = it > max_it ? it : max_it;
      tot_it += it;
      for (int i = lane; i < n; i += 64) {
        const double dqk = qn[i] - q[i];
        const double un = P.c2 * dqk - P.d1 * u[i] - P.d2 * acc[i];
        const double an = P.c0 * dqk - P.c1 * u[i] - P.c3 * acc[i];
        u[i] = un;
        acc[i] = an;
        q[i] = qn[i];
        qsn[i] = qn[i];
        // two-step first-order prediction of q_{k+3} for the chord wave
        pqn[i] = qn[i] + 2.0 * P.h * un;
        if (a.qhist && blockIdx.x == 0) a.qhist[((size_t)(k + 1) * n + i) * a.ldw + w] = qn[i];
      }
      wave_sync();
    } else if (wave == 1 && k + 1 < P.S1) {
      // ---------------- chord step k: T(q^_{k+2}) -> CB[(k+1)&1]
      double *Cn = ((k + 1) & 1) ? CB1 : CB0;
      const double *qp = (k & 1) ? pq1 : pq0;
      if (k >= 2)
        assemble_T<BW, true>(tl, n, Sl, qp, Cn, lane);
      else
        assemble_T<BW>(tl, n, Sp, qp, Cn, lane);
      wave_sync();
      if (lane == 0 && !ldlt_serial<BW>(Cn, n)) s_flags |= DEV_SINGULAR;
      wave_sync();
      if constexpr (kChord32) {
        chord_to_f32<BW>(Cn, n, ((k + 1) & 1) ? CF1 : CF0, lane);
        wave_sync();
      }
    } else if (wave == 2 && k >= 1 && k <= P.S1) {
      // ---------------- factor step k: T(q_k) -> FT[k&1]
      double *Fn = (k & 1) ? FT1 : FT0;
      const double *qk = (k & 1) ? qs1 : qs0;
      if (k >= 2)
        assemble_T<BW, true>(tl, n, Sl, qk, Fn, lane);
      else
        assemble_T<BW>(tl, n, Sp, qk, Fn, lane);
      wave_sync();
      if (lane == 0 && !ldlt_serial<BW>(Fn, n)) s_flags |= DEV_SINGULAR;
      wave_sync();
    } else if (colw && k == 0) {
      // ---------------- Q_0 = [I 0], U_0 = [0 I], w1^2 M A_0 = -[K + K_t(q0), w1 D]
      const double *F = FM + BW * bp;
      const double *Kl = KtB + BW * bp;
      double yw[BW];
#pragma unroll
      for (int t = 0; t < BW; ++t) yw[t] = 0.0;
      for (int i = 0; i < n; ++i) {
        double v = 0.0;
        if (c < n) {
          const int dlt = i - c;
          if (dlt >= 0 && dlt <= BW)
            v = -Kl[c * bp + dlt];
          else if (dlt < 0 && -dlt <= BW)
            v = -Kl[i * bp + (-dlt)];
        } else {
          const int t = (c - n) - i + BW;
          if (t >= 0 && t < W2) v = -Dwp[(size_t)i * W2 + t];
        }
#pragma unroll
        for (int t = BW; t >= 1; --t) v -= F[(i - t) * bp + t] * yw[t - 1];
#pragma unroll
        for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
        yw[0] = v;
        Yc[(size_t)i * n2] = (CT)v;
      }
#pragma unroll
      for (int t = 0; t < BW; ++t) yw[t] = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        double v = (double)Yc[(size_t)i * n2] * F[i * bp];
#pragma unroll
        for (int t = BW; t >= 1; --t) v -= F[i * bp + t] * yw[t - 1];
#pragma unroll
        for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
        yw[0] = v;
        Ac[(size_t)i * n2] = (CT)v;
        Qc[(size_t)i * n2] = (CT)((c == i) ? 1.0 : 0.0);
        Uc[(size_t)i * n2] = (CT)((c == n + i) ? 1.0 : 0.0);
      }
    } else if (colw && k >= 2) {
      // ---------------- sensitivity step k-2 -> k-1 with the factor of T(q_{k-1})
      const double *F = (((k - 1) & 1) ? FT1 : FT0) + BW * bp;
      sens_step<BW, CT>(F, Mwp, Dwp, n, n2, P.c0, P.c1, P.c2, P.c3, P.d1, P.d2, Qc, Uc, Ac, Yc);
    }
    __syncthreads();
  }
  if constexpr (!std::is_same<CT, double>::value) {
    // reduced-precision column state: Phi = [Q; U] widened to FP64
    if (colw) {
      double *Pq = a.Phi + (size_t)w * n2 * n2 + c;
      for (int i = 0; i < n; ++i) {
        Pq[(size_t)i * n2] = (double)Qc[(size_t)i * n2];
        Pq[(size_t)(n + i) * n2] = (double)Uc[(size_t)i * n2];
      }
    }
  }

  // ============================================================ epilogue
  if (wave == 0 && blockIdx.x == 0) {
    bool nan = false;
    for (int i = lane; i < n; i += 64) {
      a.zT[(size_t)i * a.ldw + w] = q[i];
      a.zT[(size_t)(n + i) * a.ldw + w] = u[i];
      if (!isfinite(q[i]) || !isfinite(u[i])) nan = true;
    }
    if (nan) atomicOr(&a.st->flags, (int)DEV_NAN);
    if (lane == 0) {
      atomicMax(&a.st->max_iters, max_it);
      atomicAdd(&a.st->total_iters, tot_it);
    }
  }
  if (threadIdx.x == 0) {
    if (s_flags) atomicOr(&a.st->flags, s_flags);
    if (s_fail_step != INT_MAX) atomicMin(&a.st->first_step, s_fail_step);
  }
}

template <int BW>
size_t fused_lds_bytes(int n, int nnz2, int nnz3) {
  constexpr bool kChord32 = BW <= 6;
  const size_t base = sizeof(double) * ((size_t)(kChord32 ? 6 : 7) * (n + BW) * (BW + 1) + 10 * ((size_t)n + 1) + 8 +
                                        nnz2 + nnz3) +
                      sizeof(int) * (2 * ((size_t)n + 1) + nnz2 + 2 * (size_t)nnz3);
  const size_t f32 = kChord32 ? sizeof(float) * 17 * (size_t)chord_rows(n) : 0;
  return ((base + 15) & ~(size_t)15) + f32;
}

template <int BW>
fse_status launch_bw(fse_ctx *ctx, int B, double *Phi, const TrajParams &P) {
  constexpr int W2 = 2 * BW + 1;
  const size_t n = ctx->n;
  const size_t band = (size_t)ctx->Bmax * n * W2;
  if (ctx->fused_band_elems < band) {
    for (double *p : {ctx->Sp, ctx->Mwp, ctx->Dwp, ctx->Kp})
      if (p) (void)hipFree(p);
    ctx->Sp = ctx->Mwp = ctx->Dwp = ctx->Kp = nullptr;
    ctx->fused_band_elems = 0;
    if (hipMalloc((void **)&ctx->Sp, sizeof(double) * band) != hipSuccess ||
        hipMalloc((void **)&ctx->Mwp, sizeof(double) * band) != hipSuccess ||
        hipMalloc((void **)&ctx->Dwp, sizeof(double) * band) != hipSuccess ||
        hipMalloc((void **)&ctx->Kp, sizeof(double) * n * W2) != hipSuccess) {
      ctx->err = "hipMalloc failed for the per-point bands";
      return FSE_E_NOMEM;
    }
    ctx->fused_band_elems = band;
  }
  const int total = B * (int)n * W2;
  hipLaunchKernelGGL(k_point_bands<BW>, dim3((total + 255) / 256), dim3(256), 0, ctx->stream, P, ctx->Mb,
                     ctx->Db, ctx->Kb, ctx->omega_d, B, ctx->Sp, ctx->Mwp, ctx->Dwp, ctx->Kp);
  FusedArgs a;
  a.P = P;
  a.Kb0 = ctx->Kb;
  a.F = ctx->F;
  a.f2_ptr = ctx->f2_ptr;
  a.f2_jk = ctx->f2_jk;
  a.f2_v = ctx->f2_v;
  a.f3_ptr = ctx->f3_ptr;
  a.f3_jkl = ctx->f3_jkl;
  a.f3_v = ctx->f3_v;
  a.f2_pk = ctx->f2_pk;
  a.f3_pk = ctx->f3_pk;
  a.nnz2 = ctx->nnz2;
  a.nnz3 = ctx->nnz3;
  a.omega = ctx->omega_d;
  a.sidx = ctx->sidx_d;
  a.Sdim = ctx->Sdim_d;
  a.q0 = ctx->qhist;
  a.u0 = ctx->u0;
  a.ldw = ctx->Wmax;
  a.zT = ctx->zTw;
  a.qhist = ctx->want_qhist ? ctx->qhist : nullptr;
  a.Phi = Phi;
  a.st = ctx->status_d;
  const size_t blk = n * 2 * n;  // one [n][2n] block
  const bool mixed = ctx->prec == FSE_PREC_MIXED_FP32;
  if (mixed) {
    // FP32 column state in the FP64 scratch: Q, U in PhiA, A, Y in sens_scr
    float *qa = reinterpret_cast<float *>(ctx->PhiA), *sa = reinterpret_cast<float *>(ctx->sens_scr);
    a.colQ = qa;
    a.colU = qa ? qa + ctx->Wmax * blk : nullptr;
    a.colA = sa;
    a.colY = sa ? sa + ctx->Wmax * blk : nullptr;
    a.colQ_ws = a.colU_ws = a.colA_ws = a.colY_ws = blk;
  } else {
    a.colQ = Phi;
    a.colU = Phi ? Phi + blk : nullptr;
    a.colQ_ws = a.colU_ws = 2 * blk;
    a.colA = ctx->PhiA;
    a.colY = ctx->sens_scr;
    a.colA_ws = a.colY_ws = blk;
  }
  const int ncw = Phi ? ctx->fused_ncw : 0;
  const int nblk = Phi ? (int)((2 * n + 64 * ncw - 1) / (64 * ncw)) : 1;
  const size_t lds = fused_lds_bytes<BW>((int)n, ctx->nnz2, ctx->nnz3);
  dim3 grid(nblk, P.W);
  if (mixed) {
    FSE_HIP(hipFuncSetAttribute((const void *)k_fused<BW, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL((k_fused<BW, float>), grid, dim3(64 * (3 + ncw)), lds, ctx->stream, a, ctx->Sp,
                       ctx->Mwp, ctx->Dwp, ctx->Kp);
  } else {
    FSE_HIP(hipFuncSetAttribute((const void *)k_fused<BW, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL((k_fused<BW, double>), grid, dim3(64 * (3 + ncw)), lds, ctx->stream, a, ctx->Sp,
                       ctx->Mwp, ctx->Dwp, ctx->Kp);
  }
  FSE_HIP(hipGetLastError());
  ctx->last_sens_launches = Phi ? 1 : 0;
  return FSE_OK;
}

int bw_bucket(int bw) { return bw <= 4 ? 4 : bw <= 6 ? 6 : bw <= 8 ? 8 : bw <= 12 ? 12 : 16; }

size_t lds_for(const fse_ctx *ctx) {
  const int n = ctx->n, a = ctx->nnz2, b = ctx->nnz3;
  switch (bw_bucket(ctx->bw)) {
    case 4: return fused_lds_bytes<4>(n, a, b);
    case 6: return fused_lds_bytes<6>(n, a, b);
    case 8: return fused_lds_bytes<8>(n, a, b);
    case 12: return fused_lds_bytes<12>(n, a, b);
    default: return fused_lds_bytes<16>(n, a, b);
  }
}

}  // namespace

int fused_band_bucket(const fse_ctx *ctx) { return bw_bucket(ctx->bw); }

bool fused_supported(const fse_ctx *ctx) {
  return ctx->bw <= 16 && ctx->n < 65536 && ctx->f2_pk && ctx->f3_pk && lds_for(ctx) + 64 <= 160 * 1024 &&
         ctx->fused_ncw >= 1 && ctx->fused_ncw <= 2;
}

fse_status launch_fused(fse_ctx *ctx, int B, double *Phi) {
  TrajParams p;
  p.n = ctx->n;
  p.bw = ctx->bw;
  p.S1 = ctx->seg_steps > 0 ? ctx->seg_steps : ctx->S1;
  p.phib = ctx->seg_phase;
  p.e = ctx->e;
  p.d = ctx->d;
  p.St = ctx->St;
  p.W = B * ctx->St;
  p.maxit = ctx->maxit;
  p.tol = ctx->tol;
  newmark_coefficients(ctx, p);
  if (Phi && !ctx->PhiA) {
    const size_t sz = sizeof(double) * ctx->Wmax * (size_t)ctx->n * 2 * ctx->n;
    if (hipMalloc((void **)&ctx->PhiA, sz) != hipSuccess || hipMalloc((void **)&ctx->sens_scr, sz) != hipSuccess) {
      ctx->err = "hipMalloc failed for the sensitivity buffers";
      return FSE_E_NOMEM;
    }
  }
  auto launch = [&]() -> fse_status {
    FSE_TRY(reset_status(ctx));
    switch (bw_bucket(ctx->bw)) {
      case 4: return launch_bw<4>(ctx, B, Phi, p);
      case 6: return launch_bw<6>(ctx, B, Phi, p);
      case 8: return launch_bw<8>(ctx, B, Phi, p);
      case 12: return launch_bw<12>(ctx, B, Phi, p);
      default: return launch_bw<16>(ctx, B, Phi, p);
    }
  };
  if (Phi && ctx->ncw_autotune) {
    // Autotuner: the first launch with sensitivities times every column-wave count (each
    // launch computes the full, identical result) and keeps the fastest for this context.
    // More column waves per work-group mean fewer work-groups per trajectory but a larger
    // work-group; which wins depends on n, the trajectory count and the CU count.
    ctx->ncw_autotune = false;
    hipEvent_t e0, e1;
    FSE_HIP(hipEventCreate(&e0));
    FSE_HIP(hipEventCreate(&e1));
    int best = ctx->fused_ncw;
    float best_ms = INFINITY;
    for (int ncw = 1; ncw <= 2; ++ncw) {
      ctx->fused_ncw = ncw;
      FSE_HIP(hipEventRecord(e0, ctx->stream));
      const fse_status st = launch();
      FSE_HIP(hipEventRecord(e1, ctx->stream));
      FSE_HIP(hipEventSynchronize(e1));
      if (st != FSE_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return st;
      }
      float ms = 0.0f;
      FSE_HIP(hipEventElapsedTime(&ms, e0, e1));
      ctx->ncw_ms[ncw - 1] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = ncw;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->fused_ncw = best;
  }
  return launch();
}
