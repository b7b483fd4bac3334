// omega_1 sensitivity for the fused path (Sec. 3.2.1, Eq. 23 with App. E): the derivative of
// the converged discrete trajectory with respect to omega_1 at fixed forcing ratios, for half
// bandwidths up to 12, using the per-point bands and the displacement history that the fused
// trajectory kernel leaves behind.
#include <cmath>

#include "band_ldlt.h"
#include "fse_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ---------------------------------------------------------------- omega_1 sensitivity
// d zbar(2 pi) / d omega_1 at fixed forcing ratios (the recursion of k_wsens in k_traj.hip:
// T Qw_{k+1} = w1^2 M (c0 Qw_k + c1 Uw_k + Aw_k) + w1 D (c2 Qw_k + Uw_k)
//              - (2 w1 c0 M + c2 D) q_{k+1} + 2 w1 M (c0 q_k + c1 u_k + a_k) + D (c2 q_k + u_k)),
// split in two for half bandwidths up to 16.  The factors of T(q_{k+1}) depend on the
// stored trajectory only, so k_wfactor computes all of them at once, one wave per (step,
// trajectory), and writes them to global memory; k_wsolve then runs the recursion, one
// work-group per trajectory: wave 0 forms the right-hand side and solves step k while
// wave 1 stages the factor and displacements of step k + 1 into the other LDS buffer.
template <int BW>
__global__ __launch_bounds__(64) void k_wfactor(TrajParams P, TensGlb tl, const double *__restrict__ Sp_all,
                                                const double *__restrict__ qhist, int ldw,
                                                double *__restrict__ Fall, DevStatus *st) {
  constexpr int bp = BW + 1, W2 = 2 * BW + 1;
  extern __shared__ double smem[];
  const int n = P.n, k = blockIdx.x, w = blockIdx.y, lane = threadIdx.x;
  const int b = w / P.St;
  const size_t fb = (size_t)(n + BW) * bp;
  double *F = smem;
  double *q = F + fb;
  for (size_t e = lane; e < fb; e += 64) F[e] = 0.0;
  for (int i = lane; i < n; i += 64) q[i] = qhist[((size_t)(k + 1) * n + i) * ldw + w];
  __syncthreads();
  [[clang::always_inline]] assemble_T<BW>(tl, n, Sp_all + (size_t)b * n * W2, q, F, lane);
  __syncthreads();
  if (lane == 0) {
    bool ok;
    [[clang::always_inline]] ok = ldlt_serial<BW>(F, n);
    if (!ok) atomicOr(&st->flags, (int)DEV_SINGULAR);
  }
  __syncthreads();
  double *out = Fall + ((size_t)w * P.S1 + k) * fb;
  for (size_t e = lane; e < fb; e += 64) out[e] = F[e];
}

template <int BW>
__global__ __launch_bounds__(128) void k_wsolve(TrajParams P, TensGlb tl, const double *__restrict__ Mb,
                                                const double *__restrict__ Db, const double *__restrict__ Kb,
                                                const double *__restrict__ Floads, const double *__restrict__ Mwp_all,
                                                const double *__restrict__ omega, const int32_t *__restrict__ sidx,
                                                const int32_t *__restrict__ Sdim, const double *__restrict__ qhist,
                                                const double *__restrict__ u0, int ldw,
                                                const double *__restrict__ Fall, double *__restrict__ dzT,
                                                DevStatus *st) {
  constexpr int bp = BW + 1, W2 = 2 * BW + 1;
  extern __shared__ double smem[];
  const int n = P.n, w = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = w / P.St, s = w - b * P.St;
  const int bw = P.bw, W2u = 2 * bw + 1;  // unpadded full rows of M, D, K
  const size_t fb = (size_t)(n + BW) * bp;
  double *FM = smem;                 // factor of w1^2 M
  double *FS0 = FM + fb;             // factors of T(q_{k+1}), double buffered
  double *FS1 = FS0 + fb;
  double *QN0 = FS1 + fb;            // q_{k+1}, double buffered
  double *QN1 = QN0 + n;
  double *q = QN1 + n;
  double *u = q + n;
  double *a = u + n;
  double *Qw = a + n;
  double *Uw = Qw + n;
  double *Aw = Uw + n;
  double *x = Aw + n;
  double *cs = x + n;
  const double *om = omega + b * P.d;
  const double w1 = om[0], w1s = w1 * w1;
  const double *__restrict__ Mwp = Mwp_all + (size_t)b * n * W2;
  const double *__restrict__ Fw = Fall + (size_t)w * P.S1 * fb;

  if (wave == 0) {
    for (size_t e = lane; e < fb; e += 64) FM[e] = 0.0;
    for (int i = lane; i < n; i += 64) {
      q[i] = qhist[(size_t)i * ldw + w];
      u[i] = u0[(size_t)i * ldw + w];
    }
    if (lane < P.e)
      cs[lane] = lane == 0 ? 1.0 : cos(kTwoPi * (double)sidx[(lane - 1) * P.St + s] / (double)Sdim[lane - 1]);
    wave_sync();
    for (int pos = lane; pos < n * bp; pos += 64) {
      const int m = pos / bp, rr = pos - m * bp, i = m + rr;
      FM[BW * bp + pos] = i < n ? Mwp[(size_t)i * W2 + (BW - rr)] : 0.0;
    }
    // consistent initial acceleration: (w1^2 M) a0 = e0 - w1 D u0 - K q0 - f_nl(q0)
    for (int i = lane; i < n; i += 64) {
      double v = 0.0;
      for (int f = 0; f < P.e; ++f) v += Floads[(size_t)f * n + i] * cs[f];
      for (int t = 0; t < W2u; ++t) {
        const int j = i - bw + t;
        if (j < 0 || j >= n) continue;
        v -= w1 * Db[(size_t)i * W2u + t] * u[j] + Kb[(size_t)i * W2u + t] * q[j];
      }
      a[i] = v - fnl_row(tl, q, i);
    }
    wave_sync();
    if (lane == 0) {
      bool ok;
      [[clang::always_inline]] ok = ldlt_serial<BW>(FM, n);
      if (!ok) atomicOr(&st->flags, (int)DEV_SINGULAR);
      [[clang::always_inline]] ldlt_solve_serial<BW>(FM, n, a);
    }
    wave_sync();
    // (w1^2 M) Aw_0 = -D u0 - 2 w1 M a0;  Qw_0 = Uw_0 = 0
    for (int i = lane; i < n; i += 64) {
      double v = 0.0;
      for (int t = 0; t < W2u; ++t) {
        const int j = i - bw + t;
        if (j < 0 || j >= n) continue;
        v -= Db[(size_t)i * W2u + t] * u[j] + 2.0 * w1 * Mb[(size_t)i * W2u + t] * a[j];
      }
      x[i] = v;
      Qw[i] = 0.0;
      Uw[i] = 0.0;
    }
    wave_sync();
    if (lane == 0) [[clang::always_inline]] ldlt_solve_serial<BW>(FM, n, x);
    wave_sync();
    for (int i = lane; i < n; i += 64) Aw[i] = x[i];
  } else {
    for (size_t e = lane; e < fb; e += 64) FS0[e] = Fw[e];
    for (int i = lane; i < n; i += 64) QN0[i] = qhist[((size_t)n + i) * ldw + w];
  }
  __syncthreads();

  for (int k = 0; k < P.S1; ++k) {
    if (wave == 1) {
      if (k + 1 < P.S1) {
        double *Fn = (k & 1) ? FS0 : FS1;
        double *Qn = (k & 1) ? QN0 : QN1;
        const double *src = Fw + (size_t)(k + 1) * fb;
        for (size_t e = lane; e < fb; e += 64) Fn[e] = src[e];
        for (int i = lane; i < n; i += 64) Qn[i] = qhist[((size_t)(k + 2) * n + i) * ldw + w];
      }
    } else {
      const double *Fk = (k & 1) ? FS1 : FS0;
      const double *qn = (k & 1) ? QN1 : QN0;
      for (int i = lane; i < n; i += 64) {
        double v = 0.0;
        for (int t = 0; t < W2u; ++t) {
          const int j = i - bw + t;
          if (j < 0 || j >= n) continue;
          const double Mij = Mb[(size_t)i * W2u + t], Dij = Db[(size_t)i * W2u + t];
          v += w1s * Mij * (P.c0 * Qw[j] + P.c1 * Uw[j] + P.c3 * Aw[j]) + w1 * Dij * (P.c2 * Qw[j] + P.d1 * Uw[j] + P.d2 * Aw[j]);
          v += -(2.0 * w1 * P.c0 * Mij + P.c2 * Dij) * qn[j] +
               2.0 * w1 * Mij * (P.c0 * q[j] + P.c1 * u[j] + P.c3 * a[j]) + Dij * (P.c2 * q[j] + P.d1 * u[j] + P.d2 * a[j]);
        }
        x[i] = v;
      }
      wave_sync();
      if (lane == 0) [[clang::always_inline]] ldlt_solve_serial<BW>(Fk, n, x);
      wave_sync();
      for (int i = lane; i < n; i += 64) {
        const double dQ = x[i] - Qw[i];
        const double uwn = P.c2 * dQ - P.d1 * Uw[i] - P.d2 * Aw[i];
        const double awn = P.c0 * dQ - P.c1 * Uw[i] - P.c3 * Aw[i];
        Qw[i] = x[i];
        Uw[i] = uwn;
        Aw[i] = awn;
        const double dqk = qn[i] - q[i];
        const double un = P.c2 * dqk - P.d1 * u[i] - P.d2 * a[i];
        const double an = P.c0 * dqk - P.c1 * u[i] - P.c3 * a[i];
        u[i] = un;
        a[i] = an;
        q[i] = qn[i];
      }
    }
    __syncthreads();
  }
  if (wave == 0) {
    bool nan = false;
    for (int i = lane; i < n; i += 64) {
      dzT[(size_t)i * ldw + w] = Qw[i];
      dzT[(size_t)(n + i) * ldw + w] = Uw[i];
      if (!isfinite(Qw[i]) || !isfinite(Uw[i])) nan = true;
    }
    if (nan) atomicOr(&st->flags, (int)DEV_NAN);
  }
}

template <int BW>
fse_status launch_wsens_bw(fse_ctx *ctx, const TrajParams &P, double *dzT) {
  constexpr int bp = BW + 1;
  const size_t n = ctx->n, fb = (n + BW) * bp;
  const size_t need = (size_t)P.W * P.S1 * fb;
  if (ctx->wfac_elems < need) {
    if (ctx->wfac) (void)hipFree(ctx->wfac);
    ctx->wfac = nullptr;
    ctx->wfac_elems = 0;
    if (hipMalloc((void **)&ctx->wfac, sizeof(double) * need) != hipSuccess) {
      ctx->err = "hipMalloc failed for the omega-sensitivity factors";
      return FSE_E_NOMEM;
    }
    ctx->wfac_elems = need;
  }
  const TensGlb tl{(glb_int *)ctx->f2_ptr, (glb_int *)ctx->f3_ptr, (glb_u32 *)ctx->f2_pk, (glb_u32 *)ctx->f3_pk,
                   (glb_double *)ctx->f2_v, (glb_double *)ctx->f3_v};
  const size_t lds_f = sizeof(double) * (fb + n);
  hipLaunchKernelGGL(k_wfactor<BW>, dim3(P.S1, P.W), dim3(64), lds_f, ctx->stream, P, tl, ctx->Sp, ctx->qhist,
                     ctx->Wmax, ctx->wfac, ctx->status_d);
  FSE_HIP(hipGetLastError());
  const size_t lds_s = sizeof(double) * (3 * fb + 9 * n + 8);
  hipLaunchKernelGGL(k_wsolve<BW>, dim3(P.W), dim3(128), lds_s, ctx->stream, P, tl, ctx->Mb, ctx->Db, ctx->Kb,
                     ctx->F, ctx->Mwp, ctx->omega_d, ctx->sidx_d, ctx->Sdim_d, ctx->qhist, ctx->u0, ctx->Wmax,
                     ctx->wfac, dzT, ctx->status_d);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

}  // namespace

fse_status launch_wsens_fused(fse_ctx *ctx, int B, double *dzT) {
  // the per-point bands it reads are those of the fused integration
  if (!fused_eligible(ctx) || wide_eligible(ctx)) return FSE_E_UNSUPPORTED;
  const int BWb = fused_band_bucket(ctx);
  const size_t fb = (size_t)(ctx->n + BWb) * (BWb + 1);
  // the per-step factors of every trajectory are held at once: stay within 8 GiB, and the
  // solve kernel's three factor buffers and vectors within the LDS
  if ((size_t)B * ctx->St > 65535 || (size_t)B * ctx->St * ctx->S1 * fb * sizeof(double) > (8ull << 30) ||
      sizeof(double) * (3 * fb + 9 * (size_t)ctx->n + 8) > 64 * 1024)
    return FSE_E_UNSUPPORTED;
  TrajParams p;
  p.n = ctx->n;
  p.bw = ctx->bw;
  p.S1 = ctx->S1;
  p.phib = 0.0;
  p.e = ctx->e;
  p.d = ctx->d;
  p.St = ctx->St;
  p.W = B * ctx->St;
  p.maxit = ctx->maxit;
  p.tol = ctx->tol;
  newmark_coefficients(ctx, p);
  switch (BWb) {
    case 4: return launch_wsens_bw<4>(ctx, p, dzT);
    case 6: return launch_wsens_bw<6>(ctx, p, dzT);
    case 8: return launch_wsens_bw<8>(ctx, p, dzT);
    case 12: return launch_wsens_bw<12>(ctx, p, dzT);
    default: return FSE_E_UNSUPPORTED;  // the register windows of BW = 16 spill: generic replay
  }
}

