// Fused trajectory kernel: state integration and sensitivity propagation of one
// trajectory in one work-group (App. E), for half bandwidths up to 16.
//
// Work-group (p, w): trajectory w, sensitivity columns [p*64*NCW, (p+1)*64*NCW).
//   wave 0      state: average-acceleration Newmark (Eqs. E4-E7); the step
//               equation (E6) is solved by a chord Newton whose matrix is the
//               factor of T(q_k) = S + K_t(q_k) from the end of the previous
//               step; after convergence T(q_{k+1}) is assembled and factored
//               (banded LDL^T with a register window) into the other buffer.
//   waves 1..   sensitivities, one step behind the state: in iteration k they
//               advance [Q; U; A] from step k-1 to k with the factor of T(q_k)
//               that wave 0 produced in iteration k-1 (exact derivative of the
//               converged discrete map, Eqs. E8-E9).
// One barrier per step separates producer and consumers (double-buffered factor).
//
// Banded data are padded to the compile-time half bandwidth BW >= bw with zeros:
//   full rows  [n][2BW+1]  entry (i, j) at [i][j - i + BW]   (global, per point)
//   LDL^T      [n][BW+1]   entry (j + r, j) at [j][r]; [j][0] holds 1 / d_j (LDS)
#include <climits>
#include <cmath>

#include "fse_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Order LDS traffic between the lanes of one wave (LDS operations of a wave are
// executed in issue order; this keeps the compiler from reordering across it).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

struct FusedArgs {
  TrajParams P;
  const double *Mb0, *Db0, *Kb0;           // unpadded full rows [n][2bw+1]
  const double *F;                         // loads [e][n]
  const int32_t *f2_ptr, *f2_jk;
  const double *f2_v;
  const int32_t *f3_ptr, *f3_jkl;
  const double *f3_v;
  const int32_t *kt_ptr, *kt_idx;
  const double *kt_c;
  const double *omega;                     // [B][d]
  const int32_t *sidx, *Sdim;
  const double *Sp, *Mwp, *Dwp;            // padded full rows [B][n][2BW+1]
  const double *q0, *u0;                   // [n][ldw]
  int ldw;
  double *zT;                              // [2n][ldw]
  double *Phi;                             // [W][2n][2n] or null
  double *PhiA;                            // [W][n][2n]
  double *Ysc;                             // [W][n][2n]
  DevStatus *st;
};

__device__ inline double fnl_row(const FusedArgs &a, const double *q, int i) {
  double f = 0.0;
  for (int p = a.f2_ptr[i]; p < a.f2_ptr[i + 1]; ++p)
    f += a.f2_v[p] * q[a.f2_jk[2 * p]] * q[a.f2_jk[2 * p + 1]];
  for (int p = a.f3_ptr[i]; p < a.f3_ptr[i + 1]; ++p)
    f += a.f3_v[p] * q[a.f3_jkl[3 * p]] * q[a.f3_jkl[3 * p + 1]] * q[a.f3_jkl[3 * p + 2]];
  return f;
}

// K_t(q)(i, m) for i >= m, i - m <= bw (lower band, runtime positions)
__device__ inline double kt_lower(const FusedArgs &a, const double *q, int m, int r) {
  const int pos = m * (a.P.bw + 1) + r;
  double v = 0.0;
  for (int p = a.kt_ptr[pos]; p < a.kt_ptr[pos + 1]; ++p) {
    const int x = a.kt_idx[2 * p], y = a.kt_idx[2 * p + 1];
    v += a.kt_c[p] * q[x] * (y >= 0 ? q[y] : 1.0);
  }
  return v;
}

// In-place banded LDL^T by one lane with a register window.  On entry F holds the
// lower band of a symmetric matrix ([m][r] = A(m+r, m)); on exit [j][0] = 1/d_j and
// [j][r] = l_{j+r, j}.  Returns false on a zero / non-finite pivot.
template <int BW>
__device__ bool ldlt_serial(double *F, int n) {
  constexpr int bp = BW + 1;
  double Wn[BW + 1][BW + 1];
#pragma unroll
  for (int r = 0; r <= BW; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) Wn[r][c] = (r < n) ? F[c * bp + (r - c)] : 0.0;
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    const double d = Wn[0][0];
    ok = ok && (d != 0.0) && isfinite(d);
    const double inv = 1.0 / d;
    double l[BW + 1];
#pragma unroll
    for (int r = 1; r <= BW; ++r) l[r] = Wn[r][0] * inv;
    F[j * bp] = inv;
#pragma unroll
    for (int r = 1; r <= BW; ++r)
      if (j + r < n) F[j * bp + r] = l[r];
#pragma unroll
    for (int r = 1; r <= BW; ++r)
#pragma unroll
      for (int c = 1; c <= r; ++c) Wn[r][c] -= Wn[r][0] * l[c];
#pragma unroll
    for (int r = 0; r < BW; ++r)
#pragma unroll
      for (int c = 0; c <= r; ++c) Wn[r][c] = Wn[r + 1][c + 1];
    const int nr = j + 1 + BW;  // new bottom row of the window
#pragma unroll
    for (int c = 0; c <= BW; ++c) Wn[BW][c] = (nr < n) ? F[(j + 1 + c) * bp + (BW - c)] : 0.0;
  }
  return ok;
}

// Solve (L D L^T) x = x in place by one lane; the term with the most recent unknown
// is applied last so each row adds one dependent FMA to the critical path.
template <int BW>
__device__ void ldlt_solve_serial(const double *F, int n, double *x) {
  constexpr int bp = BW + 1;
  double yw[BW];
#pragma unroll
  for (int t = 0; t < BW; ++t) yw[t] = 0.0;
  for (int i = 0; i < n; ++i) {
    double acc = x[i];
#pragma unroll
    for (int t = BW; t >= 1; --t)
      if (i >= t) acc -= F[(i - t) * bp + t] * yw[t - 1];
#pragma unroll
    for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
    yw[0] = acc;
    x[i] = acc;
  }
#pragma unroll
  for (int t = 0; t < BW; ++t) yw[t] = 0.0;
  for (int i = n - 1; i >= 0; --i) {
    double acc = x[i] * F[i * bp];
#pragma unroll
    for (int t = BW; t >= 1; --t) acc -= F[i * bp + t] * yw[t - 1];
#pragma unroll
    for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
    yw[0] = acc;
    x[i] = acc;
  }
}

// Per-point padded bands: S = w1^2 c0 M + w1 c2 D + K, w1^2 M, w1 D.
template <int BW>
__global__ void k_point_bands(TrajParams P, const double *__restrict__ Mb, const double *__restrict__ Db,
                              const double *__restrict__ Kb, const double *__restrict__ omega, int B,
                              double *__restrict__ Sp, double *__restrict__ Mwp, double *__restrict__ Dwp) {
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
}

template <int BW>
__global__ __launch_bounds__(256) void k_fused(FusedArgs a, const double *__restrict__ Sp_all,
                                               const double *__restrict__ Mwp_all,
                                               const double *__restrict__ Dwp_all) {
  constexpr int bp = BW + 1, W2 = 2 * BW + 1;
  extern __shared__ double smem[];
  const TrajParams &P = a.P;
  const int n = P.n, n2 = 2 * n;
  const int w = blockIdx.y;
  const int b = w / P.St, s = w - b * P.St;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ncw = (blockDim.x >> 6) - 1;
  const double *om = a.omega + b * P.d;
  const double w1 = om[0];
  // read-only per-point bands; __restrict__ lets uniform row reads use the scalar path
  const double *__restrict__ Sp = Sp_all + (size_t)b * n * W2;
  const double *__restrict__ Mwp = Mwp_all + (size_t)b * n * W2;
  const double *__restrict__ Dwp = Dwp_all + (size_t)b * n * W2;

  double *FM = smem;                     // factor of w1^2 M
  double *FT0 = FM + (size_t)n * bp;     // factors of T, double buffered
  double *FT1 = FT0 + (size_t)n * bp;
  double *KtB = FT1 + (size_t)n * bp;    // lower band of K + K_t(q0)
  double *q = KtB + (size_t)n * bp;
  double *u = q + n;
  double *acc = u + n;
  double *qn = acc + n;
  double *bv = qn + n;
  double *r = bv + n;
  double *cs = r + n;                    // forcing cosines [8]
  __shared__ int s_fail_step;
  __shared__ int s_flags;

  // ============================================================ prologue (wave 0)
  if (wave == 0) {
    if (lane == 0) {
      s_fail_step = INT_MAX;
      s_flags = 0;
    }
    for (int i = lane; i < n; i += 64) {
      q[i] = a.q0[(size_t)i * a.ldw + w];
      u[i] = a.u0[(size_t)i * a.ldw + w];
    }
    if (lane < P.e) {
      double c;
      if (lane == 0) {
        c = 1.0;
      } else {
        const double ph = kTwoPi * (double)a.sidx[(lane - 1) * P.St + s] / (double)a.Sdim[lane - 1];
        c = cos(ph);
      }
      cs[lane] = c;
    }
    wave_sync();
    // a0 right-hand side: e0 - w1 D u0 - K q0 - f_nl(q0); lower bands of w1^2 M, K + K_t(q0), T(q0)
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
      acc[i] = v - fnl_row(a, q, i);
    }
    for (int pos = lane; pos < n * bp; pos += 64) {
      const int m = pos / bp, rr = pos - m * bp, i = m + rr;
      double vm = 0.0, vk = 0.0, vt = 0.0;
      if (i < n) {
        const size_t e = (size_t)i * W2 + (BW - rr);
        const double kt = rr <= P.bw ? kt_lower(a, q, m, rr) : 0.0;
        const double kk = rr <= P.bw ? a.Kb0[(size_t)i * (2 * P.bw + 1) + (P.bw - rr)] : 0.0;
        vm = Mwp[e];
        vk = kk + kt;
        vt = Sp[e] + kt;
      }
      FM[pos] = vm;
      KtB[pos] = vk;
      FT0[pos] = vt;
    }
    wave_sync();
    if (lane == 0) {
      bool ok = ldlt_serial<BW>(FM, n);
      ldlt_solve_serial<BW>(FM, n, acc);
      ok = ldlt_serial<BW>(FT0, n) && ok;
      if (!ok) s_flags |= DEV_SINGULAR;
    }
    wave_sync();
  }
  __syncthreads();

  // ============================================================ steps
  const int c = blockIdx.x * (64 * ncw) + (wave - 1) * 64 + lane;
  const bool colw = wave >= 1 && c < n2 && a.Phi != nullptr;
  double *Qc = a.Phi ? a.Phi + (size_t)w * n2 * n2 + c : nullptr;
  double *Uc = a.Phi ? Qc + (size_t)n * n2 : nullptr;
  double *Ac = a.PhiA + (size_t)w * n * n2 + c;
  double *Yc = a.Ysc + (size_t)w * n * n2 + c;
  int max_it = 0;
  unsigned long long tot_it = 0;

  for (int k = 0; k <= P.S1; ++k) {
    if (wave == 0 && k < P.S1) {
      // ---------------- state step k: q_k -> q_{k+1}, chord matrix T(q_k) in FT[k%2]
      const double *Fc = (k & 1) ? FT1 : FT0;
      double *Fn = (k & 1) ? FT0 : FT1;
      const double phi1 = (double)(k + 1) * P.h;
      if (lane < P.e) {
        double cc;
        if (lane == 0) {
          cc = cos(phi1);
        } else {
          const double ph = kTwoPi * (double)a.sidx[(lane - 1) * P.St + s] / (double)a.Sdim[lane - 1];
          cc = cos(ph + om[lane] / w1 * phi1);
        }
        cs[lane] = cc;
      }
      wave_sync();
      for (int i = lane; i < n; i += 64) {
        double v = 0.0;
        for (int f = 0; f < P.e; ++f) v += a.F[(size_t)f * n + i] * cs[f];
#pragma unroll
        for (int t = 0; t < W2; ++t) {
          const int j = i - BW + t;
          if (j < 0 || j >= n) continue;
          v += Mwp[(size_t)i * W2 + t] * (P.c0 * q[j] + P.c1 * u[j] + acc[j]) +
               Dwp[(size_t)i * W2 + t] * (P.c2 * q[j] + u[j]);
        }
        bv[i] = v;
        qn[i] = q[i] + P.h * u[i] + 0.5 * P.h * P.h * acc[i];
      }
      wave_sync();
      double prev = INFINITY;
      bool conv = false;
      int it = 0;
      for (; it < P.maxit && !conv; ++it) {
        for (int i = lane; i < n; i += 64) {
          double v = fnl_row(a, qn, i) - bv[i];
#pragma unroll
          for (int t = 0; t < W2; ++t) {
            const int j = i - BW + t;
            if (j < 0 || j >= n) continue;
            v += Sp[(size_t)i * W2 + t] * qn[j];
          }
          r[i] = v;
        }
        wave_sync();
        if (lane == 0) ldlt_solve_serial<BW>(Fc, n, r);
        wave_sync();
        double nd = 0.0, nq = 0.0;
        for (int i = lane; i < n; i += 64) {
          const double dq = r[i];
          const double v = qn[i] - dq;
          qn[i] = v;
          nd = fmax(nd, fabs(dq));
          nq = fmax(nq, fabs(v));
        }
        nd = wave_max(nd);
        nq = wave_max(nq);
        wave_sync();
        if (!(nd == nd) || !(nq == nq)) {
          it = P.maxit;
          break;
        }
        const double tolq = P.tol * nq;
        // converged: update below tolerance; or the noise floor (update stops shrinking
        // while below 1e3 tol); or the linear-convergence bound rho/(1-rho)|dq| <= tol
        const double rho = it > 0 ? nd / prev : 1.0;
        if (nd <= tolq || (nd <= 1e3 * tolq && nd > 0.5 * prev) ||
            (rho < 0.5 && rho / (1.0 - rho) * nd <= tolq))
          conv = true;
        prev = nd;
      }
      if (!conv && lane == 0) {
        s_flags |= DEV_NOCONV;
        if (k < s_fail_step) s_fail_step = k;
      }
      max_it = it > max_it ? it : max_it;
      tot_it += it;
      for (int i = lane; i < n; i += 64) {
        const double dqk = qn[i] - q[i];
        const double un = P.c2 * dqk - u[i];
        const double an = P.c0 * dqk - P.c1 * u[i] - acc[i];
        u[i] = un;
        acc[i] = an;
        q[i] = qn[i];
      }
      wave_sync();
      // T(q_{k+1}) for the sensitivity step k and the chord of step k+1
      for (int pos = lane; pos < n * bp; pos += 64) {
        const int m = pos / bp, rr = pos - m * bp, i = m + rr;
        double vt = 0.0;
        if (i < n) vt = Sp[(size_t)i * W2 + (BW - rr)] + (rr <= P.bw ? kt_lower(a, q, m, rr) : 0.0);
        Fn[pos] = vt;
      }
      wave_sync();
      if (lane == 0) {
        if (!ldlt_serial<BW>(Fn, n)) s_flags |= DEV_SINGULAR;
      }
      wave_sync();
    }
    if (colw) {
      if (k == 0) {
        // ---------------- Q_0 = [I 0], U_0 = [0 I], w1^2 M A_0 = -[K + K_t(q0), w1 D]
        for (int i = 0; i < n; ++i) {
          double v = 0.0;
          if (c < n) {
            const int dlt = i - c;
            if (dlt >= 0 && dlt <= BW)
              v = -KtB[c * bp + dlt];
            else if (dlt < 0 && -dlt <= BW)
              v = -KtB[i * bp + (-dlt)];
          } else {
            const int cc = c - n, t = cc - i + BW;
            if (t >= 0 && t < W2) v = -Dwp[(size_t)i * W2 + t];
          }
          Yc[(size_t)i * n2] = v;
        }
        double yw[BW];
#pragma unroll
        for (int t = 0; t < BW; ++t) yw[t] = 0.0;
        for (int i = 0; i < n; ++i) {
          double v = Yc[(size_t)i * n2];
#pragma unroll
          for (int t = BW; t >= 1; --t)
            if (i >= t) v -= FM[(i - t) * bp + t] * yw[t - 1];
#pragma unroll
          for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
          yw[0] = v;
          Yc[(size_t)i * n2] = v;
        }
#pragma unroll
        for (int t = 0; t < BW; ++t) yw[t] = 0.0;
        for (int i = n - 1; i >= 0; --i) {
          double v = Yc[(size_t)i * n2] * FM[i * bp];
#pragma unroll
          for (int t = BW; t >= 1; --t) v -= FM[i * bp + t] * yw[t - 1];
#pragma unroll
          for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
          yw[0] = v;
          Ac[(size_t)i * n2] = v;
          Qc[(size_t)i * n2] = (c == i) ? 1.0 : 0.0;
          Uc[(size_t)i * n2] = (c == n + i) ? 1.0 : 0.0;
        }
      } else {
        // ---------------- sensitivity step k-1 with the factor of T(q_k) in FT[k%2]
        const double *Fk = (k & 1) ? FT1 : FT0;
        double v1w[W2], v2w[W2], yw[BW];
#pragma unroll
        for (int t = 0; t < W2; ++t) {
          const int j = t - BW;
          double Qj = 0.0, Uj = 0.0, Aj = 0.0;
          if (j >= 0 && j < n) {
            Qj = Qc[(size_t)j * n2];
            Uj = Uc[(size_t)j * n2];
            Aj = Ac[(size_t)j * n2];
          }
          v1w[t] = P.c0 * Qj + P.c1 * Uj + Aj;
          v2w[t] = P.c2 * Qj + Uj;
        }
#pragma unroll
        for (int t = 0; t < BW; ++t) yw[t] = 0.0;
        for (int i = 0; i < n; ++i) {
          const double *mr = Mwp + (size_t)i * W2;
          const double *dr = Dwp + (size_t)i * W2;
          double rhs = 0.0;
#pragma unroll
          for (int t = 0; t < W2; ++t) rhs += mr[t] * v1w[t] + dr[t] * v2w[t];
#pragma unroll
          for (int t = BW; t >= 1; --t)
            if (i >= t) rhs -= Fk[(i - t) * bp + t] * yw[t - 1];
#pragma unroll
          for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
          yw[0] = rhs;
          Yc[(size_t)i * n2] = rhs;
          // slide the windows to rows i-BW+1 .. i+BW+1
#pragma unroll
          for (int t = 0; t < W2 - 1; ++t) {
            v1w[t] = v1w[t + 1];
            v2w[t] = v2w[t + 1];
          }
          const int jn = i + BW + 1;
          double Qj = 0.0, Uj = 0.0, Aj = 0.0;
          if (jn < n) {
            Qj = Qc[(size_t)jn * n2];
            Uj = Uc[(size_t)jn * n2];
            Aj = Ac[(size_t)jn * n2];
          }
          v1w[W2 - 1] = P.c0 * Qj + P.c1 * Uj + Aj;
          v2w[W2 - 1] = P.c2 * Qj + Uj;
        }
#pragma unroll
        for (int t = 0; t < BW; ++t) yw[t] = 0.0;
        for (int i = n - 1; i >= 0; --i) {
          double x = Yc[(size_t)i * n2] * Fk[i * bp];
#pragma unroll
          for (int t = BW; t >= 1; --t) x -= Fk[i * bp + t] * yw[t - 1];
#pragma unroll
          for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
          yw[0] = x;
          const double Qo = Qc[(size_t)i * n2], Uo = Uc[(size_t)i * n2], Ao = Ac[(size_t)i * n2];
          const double dQ = x - Qo;
          Uc[(size_t)i * n2] = P.c2 * dQ - Uo;
          Ac[(size_t)i * n2] = P.c0 * dQ - P.c1 * Uo - Ao;
          Qc[(size_t)i * n2] = x;
        }
      }
    }
    __syncthreads();
  }

  // ============================================================ epilogue
  if (wave == 0) {
    bool nan = false;
    if (blockIdx.x == 0) {
      for (int i = lane; i < n; i += 64) {
        a.zT[(size_t)i * a.ldw + w] = q[i];
        a.zT[(size_t)(n + i) * a.ldw + w] = u[i];
        if (!isfinite(q[i]) || !isfinite(u[i])) nan = true;
      }
    }
    if (nan) atomicOr(&a.st->flags, (int)DEV_NAN);
    if (lane == 0 && blockIdx.x == 0) {
      if (s_flags) atomicOr(&a.st->flags, s_flags);
      if (s_fail_step != INT_MAX) atomicMin(&a.st->first_step, s_fail_step);
      atomicMax(&a.st->max_iters, max_it);
      atomicAdd(&a.st->total_iters, tot_it);
    }
  }
}

template <int BW>
fse_status launch_bw(fse_ctx *ctx, int B, double *Phi, const TrajParams &P) {
  constexpr int W2 = 2 * BW + 1;
  const size_t n = ctx->n;
  const size_t band = (size_t)ctx->Bmax * n * W2;
  if (ctx->fused_band_elems < band) {
    for (double *p : {ctx->Sp, ctx->Mwp, ctx->Dwp})
      if (p) (void)hipFree(p);
    ctx->Sp = ctx->Mwp = ctx->Dwp = nullptr;
    if (hipMalloc((void **)&ctx->Sp, sizeof(double) * band) != hipSuccess ||
        hipMalloc((void **)&ctx->Mwp, sizeof(double) * band) != hipSuccess ||
        hipMalloc((void **)&ctx->Dwp, sizeof(double) * band) != hipSuccess) {
      ctx->err = "hipMalloc failed for the per-point bands";
      return FSE_E_NOMEM;
    }
    ctx->fused_band_elems = band;
  }
  const int total = B * (int)n * W2;
  hipLaunchKernelGGL(k_point_bands<BW>, dim3((total + 255) / 256), dim3(256), 0, ctx->stream, P, ctx->Mb,
                     ctx->Db, ctx->Kb, ctx->omega_d, B, ctx->Sp, ctx->Mwp, ctx->Dwp);
  FusedArgs a;
  a.P = P;
  a.Mb0 = ctx->Mb;
  a.Db0 = ctx->Db;
  a.Kb0 = ctx->Kb;
  a.F = ctx->F;
  a.f2_ptr = ctx->f2_ptr;
  a.f2_jk = ctx->f2_jk;
  a.f2_v = ctx->f2_v;
  a.f3_ptr = ctx->f3_ptr;
  a.f3_jkl = ctx->f3_jkl;
  a.f3_v = ctx->f3_v;
  a.kt_ptr = ctx->kt_ptr;
  a.kt_idx = ctx->kt_idx;
  a.kt_c = ctx->kt_c;
  a.omega = ctx->omega_d;
  a.sidx = ctx->sidx_d;
  a.Sdim = ctx->Sdim_d;
  a.Sp = ctx->Sp;
  a.Mwp = ctx->Mwp;
  a.Dwp = ctx->Dwp;
  a.q0 = ctx->qhist;
  a.u0 = ctx->u0;
  a.ldw = ctx->Wmax;
  a.zT = ctx->zTw;
  a.Phi = Phi;
  a.PhiA = ctx->PhiA;
  a.Ysc = ctx->sens_scr;
  a.st = ctx->status_d;
  int ncw = 0, nblk = 1;
  if (Phi) {
    ncw = ctx->fused_ncw;
    const int cols = 64 * ncw;
    nblk = (int)((2 * n + cols - 1) / cols);
  }
  const size_t lds = sizeof(double) * ((size_t)4 * n * (BW + 1) + 7 * n + 8);
  dim3 grid(nblk, P.W);
  hipLaunchKernelGGL(k_fused<BW>, grid, dim3(64 * (1 + ncw)), lds, ctx->stream, a, ctx->Sp, ctx->Mwp,
                     ctx->Dwp);
  FSE_HIP(hipGetLastError());
  ctx->last_sens_launches = Phi ? 1 : 0;
  return FSE_OK;
}

}  // namespace

static int bw_bucket(int bw) { return bw <= 4 ? 4 : bw <= 6 ? 6 : bw <= 8 ? 8 : bw <= 12 ? 12 : 16; }

bool fused_supported(const fse_ctx *ctx) {
  if (ctx->bw > 16) return false;
  const size_t lds = sizeof(double) * ((size_t)4 * ctx->n * (bw_bucket(ctx->bw) + 1) + 7 * ctx->n + 8);
  return lds <= 64 * 1024;
}

fse_status launch_fused(fse_ctx *ctx, int B, double *Phi) {
  const TrajParams P = [&] {
    TrajParams p;
    p.n = ctx->n;
    p.bw = ctx->bw;
    p.S1 = ctx->S1;
    p.e = ctx->e;
    p.d = ctx->d;
    p.St = ctx->St;
    p.W = B * ctx->St;
    p.maxit = ctx->maxit;
    p.tol = ctx->tol;
    p.h = 2.0 * M_PI / ctx->S1;
    p.c0 = 4.0 / (p.h * p.h);
    p.c1 = 4.0 / p.h;
    p.c2 = 2.0 / p.h;
    return p;
  }();
  if (Phi && !ctx->PhiA) {
    const size_t sz = sizeof(double) * ctx->Wmax * (size_t)ctx->n * 2 * ctx->n;
    if (hipMalloc((void **)&ctx->PhiA, sz) != hipSuccess || hipMalloc((void **)&ctx->sens_scr, sz) != hipSuccess) {
      ctx->err = "hipMalloc failed for the sensitivity buffers";
      return FSE_E_NOMEM;
    }
  }
  FSE_TRY(reset_status(ctx));
  if (ctx->bw <= 4) return launch_bw<4>(ctx, B, Phi, P);
  if (ctx->bw <= 6) return launch_bw<6>(ctx, B, Phi, P);
  if (ctx->bw <= 8) return launch_bw<8>(ctx, B, Phi, P);
  if (ctx->bw <= 12) return launch_bw<12>(ctx, B, Phi, P);
  return launch_bw<16>(ctx, B, Phi, P);
}
