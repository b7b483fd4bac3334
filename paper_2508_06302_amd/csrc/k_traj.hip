// Trajectory kernels of FSE-Shooting on gfx950 (Sec. 3.3 steps 2-5, App. E).
//
// Layouts (W = B * S~ trajectories, trajectory index w = b * S~ + s, arrays
// strided by Wmax so that consecutive trajectories are contiguous):
//   qhist [S1+1][n][Wmax]   displacement history written by the state kernel
//   u0    [n][Wmax]         initial velocities u = dq/dphi_1
//   zTw   [2n][Wmax]        terminal samples [q; u](2 pi)
//   Phi   [W][2n][2n]       [Q; U] sensitivities (rows), columns fastest
//   PhiA  [W][n][2n]        A = dQ''/dz0 (Newmark acceleration sensitivities)
// Banded matrices are stored as full rows [n][2bw+1] (entry (i,j) at
// [i][j-i+bw]); a banded LDL^T factor is stored by columns [n][bw+1] with
// entry (j+r, j) at [j][r] (r = 0 holds the pivot d_j).
#include <climits>
#include <cmath>

#include "fse_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ inline double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// max over the block; red must hold blockDim.x / 64 doubles; all threads get the result
__device__ double block_max(double v, double *red) {
  v = warp_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

__device__ inline void pair_rc(int p, int &r, int &c) {
  int rr = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
  while (rr * (rr - 1) / 2 > p) --rr;
  while ((rr + 1) * rr / 2 <= p) ++rr;
  r = rr;
  c = p - rr * (rr - 1) / 2 + 1;
}

// In-place banded LDL^T of the lower band Lf (column storage, see file header),
// cooperative over the block; right-looking, one barrier per column.
__device__ void band_ldlt(double *Lf, int n, int bw, DevStatus *st) {
  const int bp = bw + 1;
  const int npairs = bw * (bw + 1) / 2;
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    const double dj = Lf[j * bp];
    if (!(dj != 0.0) || !isfinite(dj)) bad = true;
    const double inv = 1.0 / dj;
    for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
      int r, c;
      pair_rc(p, r, c);
      if (j + r < n) Lf[(j + c) * bp + (r - c)] -= Lf[j * bp + r] * Lf[j * bp + c] * inv;
    }
    __syncthreads();
    for (int r = 1 + threadIdx.x; r <= bw; r += blockDim.x)
      if (j + r < n) Lf[j * bp + r] *= inv;
  }
  __syncthreads();
  if (bad && threadIdx.x == 0) atomicOr(&st->flags, (int)DEV_SINGULAR);
}

// Solve L D L^T x = r for one right-hand side held in x (in place), executed by
// thread 0 (band factor and x in block-shared memory).
__device__ void band_solve_serial(const double *Lf, int n, int bw, double *x) {
  const int bp = bw + 1;
  for (int i = 0; i < n; ++i) {
    double y = x[i];
    const int t0 = i < bw ? i : bw;
    for (int t = t0; t >= 1; --t) y -= Lf[(i - t) * bp + t] * x[i - t];
    x[i] = y;
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = x[i] / Lf[i * bp];
    const int t1 = (n - 1 - i) < bw ? (n - 1 - i) : bw;
    for (int t = t1; t >= 1; --t) v -= Lf[i * bp + t] * x[i + t];
    x[i] = v;
  }
}

// Block-cooperative version for wide bands: every row's dot product is split over the block.
__device__ void band_solve_block(const double *Lf, int n, int bw, double *x, double *red) {
  const int bp = bw + 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < n; ++i) {
    double part = 0.0;
    const int t0 = i < bw ? i : bw;
    for (int t = 1 + threadIdx.x; t <= t0; t += blockDim.x) part += Lf[(i - t) * bp + t] * x[i - t];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += red[k];
      x[i] -= s;
    }
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {
    double part = 0.0;
    const int t1 = (n - 1 - i) < bw ? (n - 1 - i) : bw;
    for (int t = 1 + threadIdx.x; t <= t1; t += blockDim.x) part += Lf[i * bp + t] * x[i + t];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += red[k];
      x[i] = x[i] / Lf[i * bp] - s;
    }
    __syncthreads();
  }
}

__device__ inline void band_solve(const double *Lf, int n, int bw, double *x, double *red) {
  if (bw <= 24) {
    if (threadIdx.x == 0) band_solve_serial(Lf, n, bw, x);
    __syncthreads();
  } else {
    band_solve_block(Lf, n, bw, x, red);
  }
}

struct SysDev {
  const double *Mb, *Db, *Kb, *F;
  const int32_t *f2_ptr, *f2_jk;
  const double *f2_v;
  const int32_t *f3_ptr, *f3_jkl;
  const double *f3_v;
  const int32_t *kt_ptr, *kt_idx;
  const double *kt_c;
  const int32_t *ct_ptr, *ct_idx;  // C_t = d f / d qdot lists, or null (forces of q only)
  const double *ct_c;
  const int32_t *cn_ptr;  // unilateral contacts by DOF, or null
  const double *cn_v;     // (direction, gap, stiffness) per contact
  int bw, n;
};

// y = [q; qdot]: factor index j < n is q_j, j >= n is qdot_{j-n} (qd is read only then)
__device__ inline double yv(const double *q, const double *qd, int n, int j) { return j < n ? q[j] : qd[j - n]; }

// f_nl(q, qdot)_i = sum t2 y_j y_k + sum t3 y_j y_k y_l (row i of the CSR-by-output tensors)
__device__ inline double fnl_row(const SysDev &sy, const double *q, const double *qd, int i) {
  double f = 0.0;
  const int n = sy.n;
  for (int p = sy.f2_ptr[i]; p < sy.f2_ptr[i + 1]; ++p)
    f += sy.f2_v[p] * yv(q, qd, n, sy.f2_jk[2 * p]) * yv(q, qd, n, sy.f2_jk[2 * p + 1]);
  for (int p = sy.f3_ptr[i]; p < sy.f3_ptr[i + 1]; ++p)
    f += sy.f3_v[p] * yv(q, qd, n, sy.f3_jkl[3 * p]) * yv(q, qd, n, sy.f3_jkl[3 * p + 1]) *
         yv(q, qd, n, sy.f3_jkl[3 * p + 2]);
  if (sy.cn_ptr)  // a closed contact pushes back with s k (s q_i - g)
    for (int p = sy.cn_ptr[i]; p < sy.cn_ptr[i + 1]; ++p) {
      const double sg = sy.cn_v[3 * p], pen = sg * q[i] - sy.cn_v[3 * p + 1];
      if (pen > 0.0) f += sg * sy.cn_v[3 * p + 2] * pen;
    }
  return f;
}

// one tangent list at lower-band position pos = m*(bw+1) + (i-m)
__device__ inline double tangent_list(const int32_t *ptr, const int32_t *idx, const double *cf, int n,
                                      const double *q, const double *qd, int pos) {
  double v = 0.0;
  for (int p = ptr[pos]; p < ptr[pos + 1]; ++p) {
    const int a = idx[2 * p], b = idx[2 * p + 1];
    v += cf[p] * yv(q, qd, n, a) * (b >= 0 ? yv(q, qd, n, b) : 1.0);
  }
  return v;
}

// K_t(q, qdot) and C_t(q, qdot) (zero for forces of q only)
// K_t includes the generalised derivative of the contacts: k on the diagonal of a closed one.
__device__ inline double kt_entry(const SysDev &sy, const double *q, const double *qd, int pos) {
  double v = tangent_list(sy.kt_ptr, sy.kt_idx, sy.kt_c, sy.n, q, qd, pos);
  if (sy.cn_ptr) {
    const int bp = sy.bw + 1, m = pos / bp;
    if (pos == m * bp)
      for (int p = sy.cn_ptr[m]; p < sy.cn_ptr[m + 1]; ++p)
        if (sy.cn_v[3 * p] * q[m] - sy.cn_v[3 * p + 1] > 0.0) v += sy.cn_v[3 * p + 2];
  }
  return v;
}
__device__ inline double ct_entry(const SysDev &sy, const double *q, const double *qd, int pos) {
  return sy.ct_ptr ? tangent_list(sy.ct_ptr, sy.ct_idx, sy.ct_c, sy.n, q, qd, pos) : 0.0;
}

// Forcing cosines at phi_1 for sample s (Eq. E1): forcing 0 has argument phi_1,
// forcing f >= 1 has phi_{f+1,s} + rho_{f+1} phi_1.
__device__ inline double forcing_cos(int f, double phi1, const double *om, const int32_t *sidx,
                                     const int32_t *Sdim, int St, int s, double phi0) {
  if (f == 0) return cos(phi0 + phi1);
  const double ph = kTwoPi * (double)sidx[(f - 1) * St + s] / (double)Sdim[f - 1];
  return cos(ph + om[f] / om[0] * phi1);
}

__global__ void k_reset_status(DevStatus *st, int first_step) {
  if (threadIdx.x == 0) {
    st->flags = 0;
    st->first_step = first_step;
    st->max_iters = 0;
    st->pad = 0;
    st->total_iters = 0ull;
  }
}

// ------------------------------------------------------------------------ inverse DFT (Eq. 20)
__global__ void k_idft(const double *__restrict__ Z0, const double *__restrict__ G, int n, int U,
                       int St, int W, int ldw, double *__restrict__ q0, double *__restrict__ u0) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;  // state row 0..2n-1
  if (w >= W) return;
  const int b = w / St, s = w - (w / St) * St;
  const double *z = Z0 + ((size_t)b * 2 * n + i) * U;
  const double *g = G + (size_t)s * U;
  double v = 0.0;
  for (int l = 0; l < U; ++l) v += g[l] * z[l];
  if (i < n)
    q0[(size_t)i * ldw + w] = v;
  else
    u0[(size_t)(i - n) * ldw + w] = v;
}

// ------------------------------------------------------------------------ state integration
// One block per trajectory: average-acceleration Newmark (Eqs. E4-E7) with full-tangent
// Newton on Eq. (E6) at every step.  Writes the displacement history for the
// sensitivity kernel and the terminal state.
template <bool LDS>
__global__ void k_state(TrajParams P, SysDev sy, const double *__restrict__ omega,
                        const int32_t *__restrict__ sidx, const int32_t *__restrict__ Sdim,
                        double *__restrict__ qhist, double *__restrict__ uhist, const double *__restrict__ u0,
                        double *__restrict__ zT, int ldw, double *__restrict__ gscr,
                        DevStatus *st) {
  extern __shared__ double smem[];
  const int n = P.n, bw = P.bw, bp = bw + 1, w = blockIdx.x;
  const size_t stride = (size_t)n * bp + 9 * (size_t)n + 80;
  double *base = LDS ? smem : gscr + (size_t)w * stride;
  double *Lf = base;
  double *q = Lf + (size_t)n * bp;
  double *u = q + n;
  double *a = u + n;
  double *qn = a + n;
  double *bv = qn + n;
  double *r = bv + n;
  double *cs = r + 2 * n;        // e cosines (<= 8)
  double *red = cs + 8;          // block reduction scratch (<= 64)
  double *qd = red + 72;         // qdot = w1 u of the current iterate (velocity-dependent forces)
  const bool vel = sy.ct_ptr != nullptr;
  const int b = w / P.St, s = w - b * P.St;
  const double *om = omega + b * P.d;
  const double w1 = om[0];
  const double w1s = w1 * w1;
  const int W2 = 2 * bw + 1;
  const int tid = threadIdx.x, nt = blockDim.x;

  for (int i = tid; i < n; i += nt) {
    q[i] = qhist[(size_t)i * ldw + w];
    u[i] = u0[(size_t)i * ldw + w];
    if (vel) {
      qd[i] = w1 * u[i];
      uhist[(size_t)i * ldw + w] = u[i];
    }
  }
  if (tid < P.e) cs[tid] = forcing_cos(tid, 0.0, om, sidx, Sdim, P.St, s, P.phib * b);
  __syncthreads();
  // consistent initial acceleration: (w1^2 M) a0 = e0 - w1 D u0 - K q0 - f_nl(q0)
  for (int i = tid; i < n; i += nt) {
    double v = 0.0;
    for (int f = 0; f < P.e; ++f) v += sy.F[(size_t)f * n + i] * cs[f];
    const int j0 = i - bw;
    for (int t = 0; t < W2; ++t) {
      const int j = j0 + t;
      if (j < 0 || j >= n) continue;
      v -= w1 * sy.Db[(size_t)i * W2 + t] * u[j] + sy.Kb[(size_t)i * W2 + t] * q[j];
    }
    a[i] = v - fnl_row(sy, q, qd, i);
  }
  for (int pos = tid; pos < n * bp; pos += nt) {
    const int m = pos / bp, t = pos - m * bp, i = m + t;
    Lf[pos] = i < n ? w1s * sy.Mb[(size_t)i * W2 + (bw - t)] : 0.0;
  }
  __syncthreads();
  band_ldlt(Lf, n, bw, st);
  band_solve(Lf, n, bw, a, red);

  int max_it = 0;
  unsigned long long tot_it = 0;
  bool failed = false;
  for (int k = 0; k < P.S1; ++k) {
    const double phi1 = (double)(k + 1) * P.h;
    if (tid < P.e) cs[tid] = forcing_cos(tid, phi1, om, sidx, Sdim, P.St, s, P.phib * b);
    __syncthreads();
    // b_k (Eq. E7) and the predictor
    for (int i = tid; i < n; i += nt) {
      double v = 0.0;
      for (int f = 0; f < P.e; ++f) v += sy.F[(size_t)f * n + i] * cs[f];
      const int j0 = i - bw;
      for (int t = 0; t < W2; ++t) {
        const int j = j0 + t;
        if (j < 0 || j >= n) continue;
        v += w1s * sy.Mb[(size_t)i * W2 + t] * (P.c0 * q[j] + P.c1 * u[j] + P.c3 * a[j]) +
             w1 * sy.Db[(size_t)i * W2 + t] * (P.c2 * q[j] + P.d1 * u[j] + P.d2 * a[j]);
      }
      bv[i] = v;
      qn[i] = q[i] + P.h * u[i] + 0.5 * P.h * P.h * a[i];
    }
    __syncthreads();
    double prev = INFINITY;
    bool conv = false;
    int it = 0;
    for (; it < P.maxit && !conv; ++it) {
      // residual r = S qn + f_nl(qn, qdot) - b and tangent band S + K_t + w1 c2 C_t, with
      // qdot = w1 u_{k+1}(qn) for velocity-dependent forces
      if (vel) {
        for (int i = tid; i < n; i += nt)
          qd[i] = w1 * (P.c2 * (qn[i] - q[i]) - P.d1 * u[i] - P.d2 * a[i]);
        __syncthreads();
      }
      for (int i = tid; i < n; i += nt) {
        double v = -bv[i] + fnl_row(sy, qn, qd, i);
        const int j0 = i - bw;
        for (int t = 0; t < W2; ++t) {
          const int j = j0 + t;
          if (j < 0 || j >= n) continue;
          const double sij = w1s * P.c0 * sy.Mb[(size_t)i * W2 + t] +
                             w1 * P.c2 * sy.Db[(size_t)i * W2 + t] + sy.Kb[(size_t)i * W2 + t];
          v += sij * qn[j];
        }
        r[i] = v;
      }
      for (int pos = tid; pos < n * bp; pos += nt) {
        const int m = pos / bp, t = pos - m * bp, i = m + t;
        double v = 0.0;
        if (i < n) {
          const size_t e = (size_t)i * W2 + (bw - t);
          v = w1s * P.c0 * sy.Mb[e] + w1 * P.c2 * sy.Db[e] + sy.Kb[e] + kt_entry(sy, qn, qd, pos);
          if (vel) v += w1 * P.c2 * ct_entry(sy, qn, qd, pos);
        }
        Lf[pos] = v;
      }
      __syncthreads();
      band_ldlt(Lf, n, bw, st);
      band_solve(Lf, n, bw, r, red);
      double nd = 0.0, nq = 0.0;
      for (int i = tid; i < n; i += nt) {
        const double dq = r[i];
        const double v = qn[i] - dq;
        qn[i] = v;
        nd = fmax(nd, fabs(dq));
        nq = fmax(nq, fabs(v));
      }
      nd = block_max(nd, red);
      nq = block_max(nq, red);
      if (!(nd == nd) || !(nq == nq)) break;
      if (nd <= P.tol * nq || (nd <= 1e3 * P.tol * nq && nd > 0.5 * prev)) conv = true;
      prev = nd;
    }
    if (!conv && !failed) {
      failed = true;
      if (tid == 0) {
        atomicOr(&st->flags, (int)DEV_NOCONV);
        atomicMin(&st->first_step, k);
      }
    }
    max_it = it > max_it ? it : max_it;
    tot_it += it;
    // Eq. (E5) and the history for the sensitivity pass
    for (int i = tid; i < n; i += nt) {
      const double dqk = qn[i] - q[i];
      const double un = P.c2 * dqk - P.d1 * u[i] - P.d2 * a[i];
      const double an = P.c0 * dqk - P.c1 * u[i] - P.c3 * a[i];
      u[i] = un;
      a[i] = an;
      q[i] = qn[i];
      qhist[((size_t)(k + 1) * n + i) * ldw + w] = qn[i];
      if (vel) uhist[((size_t)(k + 1) * n + i) * ldw + w] = un;
    }
    __syncthreads();
  }
  bool nan = false;
  for (int i = tid; i < n; i += nt) {
    zT[(size_t)i * ldw + w] = q[i];
    zT[(size_t)(n + i) * ldw + w] = u[i];
    if (!isfinite(q[i]) || !isfinite(u[i])) nan = true;
  }
  if (nan) atomicOr(&st->flags, (int)DEV_NAN);
  if (tid == 0) {
    atomicMax(&st->max_iters, max_it);
    atomicAdd(&st->total_iters, tot_it);
  }
}

// ------------------------------------------------------------------------ sensitivities
// Exact derivative of the converged discrete map (Eqs. E8-E9): with T = S + K_t(q_{k+1})
//   T Q_{k+1} = w1^2 M (c0 Q_k + c1 U_k + A_k) + w1 D (c2 Q_k + U_k)
//   U_{k+1} = c2 (Q_{k+1} - Q_k) - U_k,  A_{k+1} = c0 (Q_{k+1} - Q_k) - c1 U_k - A_k
// Q_0 = [I 0], U_0 = [0 I], A_0 = -(w1^2 M)^-1 [K + K_t(q_0), w1 D].
// Block (p, w): columns p*blockDim.x + tid of trajectory w; the band factor of T
// is computed once per step per block, every thread sweeps its column.
template <bool LDS>
__global__ void k_sens(TrajParams P, SysDev sy, const double *__restrict__ omega,
                       const double *__restrict__ qhist, const double *__restrict__ uhist, int ldw,
                       double *__restrict__ PhiQU,
                       double *__restrict__ PhiA, double *__restrict__ Ysc,
                       double *__restrict__ gscr, DevStatus *st) {
  extern __shared__ double smem[];
  const int n = P.n, bw = P.bw, bp = bw + 1, n2 = 2 * n, W2 = 2 * bw + 1;
  const int w = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = c < n2;
  const size_t stride = (size_t)3 * n * bp + 2 * n + 8;
  double *base = LDS ? smem : gscr + ((size_t)w * gridDim.x + blockIdx.x) * stride;
  double *Lf = base;
  double *Kt = Lf + (size_t)n * bp;
  double *Ct = Kt + (size_t)n * bp;   // C_t lower band (velocity-dependent forces)
  double *qv = Ct + (size_t)n * bp;
  double *qdv = qv + n;               // qdot = w1 u of the replayed state
  const bool vel = sy.ct_ptr != nullptr;
  const int b = w / P.St;
  const double w1 = omega[b * P.d];
  const double w1s = w1 * w1;
  double *Qc = PhiQU + (size_t)w * n2 * n2 + c;
  double *Uc = Qc + (size_t)n * n2;
  double *Ac = PhiA + (size_t)w * n * n2 + c;
  double *Yc = Ysc + (size_t)w * n * n2 + c;
  const int tid = threadIdx.x, nt = blockDim.x;

  // ---- initial sensitivities
  for (int i = tid; i < n; i += nt) {
    qv[i] = qhist[(size_t)i * ldw + w];
    if (vel) qdv[i] = w1 * uhist[(size_t)i * ldw + w];
  }
  __syncthreads();
  for (int pos = tid; pos < n * bp; pos += nt) {
    const int m = pos / bp, t = pos - m * bp, i = m + t;
    Lf[pos] = i < n ? w1s * sy.Mb[(size_t)i * W2 + (bw - t)] : 0.0;
    Kt[pos] = i < n ? kt_entry(sy, qv, qdv, pos) : 0.0;
    Ct[pos] = (i < n && vel) ? ct_entry(sy, qv, qdv, pos) : 0.0;
  }
  __syncthreads();
  band_ldlt(Lf, n, bw, st);
  if (active) {
    // right-hand side column: -(K + K_t(q0)) e_c or -w1 D e_{c-n}
    for (int i = 0; i < n; ++i) {
      double v = 0.0;
      if (c < n) {
        if (abs(i - c) <= bw) {
          v = -sy.Kb[(size_t)i * W2 + (c - i + bw)];
          v -= i >= c ? Kt[c * bp + (i - c)] : Kt[i * bp + (c - i)];
        }
      } else {
        const int cc = c - n;
        if (abs(i - cc) <= bw) {
          v = -w1 * sy.Db[(size_t)i * W2 + (cc - i + bw)];
          v -= w1 * (i >= cc ? Ct[cc * bp + (i - cc)] : Ct[i * bp + (cc - i)]);
        }
      }
      Yc[(size_t)i * n2] = v;
    }
    for (int i = 0; i < n; ++i) {
      double y = Yc[(size_t)i * n2];
      const int t0 = i < bw ? i : bw;
      for (int t = 1; t <= t0; ++t) y -= Lf[(i - t) * bp + t] * Yc[(size_t)(i - t) * n2];
      Yc[(size_t)i * n2] = y;
    }
    for (int i = n - 1; i >= 0; --i) {
      double x = Yc[(size_t)i * n2] / Lf[i * bp];
      const int t1 = (n - 1 - i) < bw ? (n - 1 - i) : bw;
      for (int t = 1; t <= t1; ++t) x -= Lf[i * bp + t] * Ac[(size_t)(i + t) * n2];
      Ac[(size_t)i * n2] = x;
      Qc[(size_t)i * n2] = (c == i) ? 1.0 : 0.0;
      Uc[(size_t)i * n2] = (c == n + i) ? 1.0 : 0.0;
    }
  }
  __syncthreads();

  // ---- steps
  for (int k = 0; k < P.S1; ++k) {
    for (int i = tid; i < n; i += nt) {
      qv[i] = qhist[((size_t)(k + 1) * n + i) * ldw + w];
      if (vel) qdv[i] = w1 * uhist[((size_t)(k + 1) * n + i) * ldw + w];
    }
    __syncthreads();
    for (int pos = tid; pos < n * bp; pos += nt) {
      const int m = pos / bp, t = pos - m * bp, i = m + t;
      double v = 0.0;
      if (i < n) {
        const size_t e = (size_t)i * W2 + (bw - t);
        v = w1s * P.c0 * sy.Mb[e] + w1 * P.c2 * sy.Db[e] + sy.Kb[e] + kt_entry(sy, qv, qdv, pos);
        if (vel) {
          const double ct = ct_entry(sy, qv, qdv, pos);
          Ct[pos] = ct;
          v += w1 * P.c2 * ct;
        }
      }
      Lf[pos] = v;
    }
    __syncthreads();
    band_ldlt(Lf, n, bw, st);
    if (active) {
      for (int i = 0; i < n; ++i) {
        double rhs = 0.0;
        const int j0 = i - bw;
        for (int t = 0; t < W2; ++t) {
          const int j = j0 + t;
          if (j < 0 || j >= n) continue;
          const double Qj = Qc[(size_t)j * n2], Uj = Uc[(size_t)j * n2], Aj = Ac[(size_t)j * n2];
          // velocity-dependent forces linearise into the state-dependent damping D + C_t
          const double dij = sy.Db[(size_t)i * W2 + t] +
                             (vel ? (j <= i ? Ct[j * bp + (i - j)] : Ct[i * bp + (j - i)]) : 0.0);
          rhs += w1s * sy.Mb[(size_t)i * W2 + t] * (P.c0 * Qj + P.c1 * Uj + P.c3 * Aj) +
                 w1 * dij * (P.c2 * Qj + P.d1 * Uj + P.d2 * Aj);
        }
        const int t0 = i < bw ? i : bw;
        for (int t = 1; t <= t0; ++t) rhs -= Lf[(i - t) * bp + t] * Yc[(size_t)(i - t) * n2];
        Yc[(size_t)i * n2] = rhs;
      }
      for (int i = n - 1; i >= 0; --i) {
        double x = Yc[(size_t)i * n2] / Lf[i * bp];
        const int t1 = (n - 1 - i) < bw ? (n - 1 - i) : bw;
        for (int t = 1; t <= t1; ++t) x -= Lf[i * bp + t] * Yc[(size_t)(i + t) * n2];
        Yc[(size_t)i * n2] = x;
        const double Qo = Qc[(size_t)i * n2], Uo = Uc[(size_t)i * n2], Ao = Ac[(size_t)i * n2];
        const double dQ = x - Qo;
        Uc[(size_t)i * n2] = P.c2 * dQ - P.d1 * Uo - P.d2 * Ao;
        Ac[(size_t)i * n2] = P.c0 * dQ - P.c1 * Uo - P.c3 * Ao;
        Qc[(size_t)i * n2] = x;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------ omega_1 sensitivity
// d zbar(2 pi) / d omega_1 with the forcing frequency ratios held (frequency conditions of
// Sec. 3.2.1): the forcing is then a fixed function of phi_1 and omega_1 enters Eq. (E1) only
// through w1^2 M and w1 D.  Exact derivative of the converged discrete map (Eqs. E4-E7):
//   T Qw_{k+1} = w1^2 M (c0 Qw_k + c1 Uw_k + Aw_k) + w1 D (c2 Qw_k + Uw_k)
//                - (2 w1 c0 M + c2 D) q_{k+1} + 2 w1 M (c0 q_k + c1 u_k + a_k) + D (c2 q_k + u_k)
//   Uw_{k+1} = c2 (Qw_{k+1} - Qw_k) - Uw_k,  Aw_{k+1} = c0 (Qw_{k+1} - Qw_k) - c1 Uw_k - Aw_k
// with T = S + K_t(q_{k+1}), Qw_0 = Uw_0 = 0 and w1^2 M Aw_0 = -D u_0 - 2 w1 M a_0 (the
// derivative of the consistent initial acceleration).  One block per trajectory; the state is
// replayed from the displacement history of the integration, so the derivative is that of the
// very trajectory whose end point enters R.  Output dzT [2n][ldw] = [Qw; Uw](2 pi).
// entry (i, j) of a symmetric matrix from its lower band (pos = m (bw+1) + (i - m), m <= i)
__device__ inline double ct_band(const double *Cb, int bp, int i, int j) {
  return i >= j ? Cb[j * bp + (i - j)] : Cb[i * bp + (j - i)];
}

template <bool LDS>
__global__ void k_wsens(TrajParams P, SysDev sy, const double *__restrict__ omega,
                        const int32_t *__restrict__ sidx, const int32_t *__restrict__ Sdim,
                        const double *__restrict__ qhist, const double *__restrict__ u0, int ldw,
                        double *__restrict__ dzT, double *__restrict__ gscr, DevStatus *st) {
  extern __shared__ double smem[];
  const int n = P.n, bw = P.bw, bp = bw + 1, w = blockIdx.x;
  const bool vel = sy.ct_ptr != nullptr;
  const size_t stride = (size_t)n * bp + 8 * (size_t)n + 80 + (vel ? (size_t)n * bp + n : 0);
  double *base = LDS ? smem : gscr + (size_t)w * stride;
  double *Lf = base;
  double *q = Lf + (size_t)n * bp;
  double *u = q + n;
  double *a = u + n;
  double *qn = a + n;
  double *Qw = qn + n;
  double *Uw = Qw + n;
  double *Aw = Uw + n;
  double *x = Aw + n;
  double *cs = x + n;            // e cosines (<= 8)
  double *red = cs + 8;          // block reduction scratch (<= 64)
  // velocity-dependent forces: C_t lower band and qdot = w1 u of the current state
  double *Ct = red + 72;
  double *qd = Ct + (size_t)n * bp;
  const int b = w / P.St, s = w - b * P.St;
  const double *om = omega + b * P.d;
  const double w1 = om[0];
  const double w1s = w1 * w1;
  const int W2 = 2 * bw + 1;
  const int tid = threadIdx.x, nt = blockDim.x;

  for (int i = tid; i < n; i += nt) {
    q[i] = qhist[(size_t)i * ldw + w];
    u[i] = u0[(size_t)i * ldw + w];
    if (vel) qd[i] = w1 * u[i];
  }
  if (tid < P.e) cs[tid] = forcing_cos(tid, 0.0, om, sidx, Sdim, P.St, s, P.phib * b);
  __syncthreads();
  // consistent initial acceleration (w1^2 M) a0 = e0 - w1 D u0 - K q0 - f_nl(q0)
  for (int i = tid; i < n; i += nt) {
    double v = 0.0;
    for (int f = 0; f < P.e; ++f) v += sy.F[(size_t)f * n + i] * cs[f];
    for (int t = 0; t < W2; ++t) {
      const int j = i - bw + t;
      if (j < 0 || j >= n) continue;
      v -= w1 * sy.Db[(size_t)i * W2 + t] * u[j] + sy.Kb[(size_t)i * W2 + t] * q[j];
    }
    a[i] = v - fnl_row(sy, q, vel ? qd : q, i);  // without velocity forces the qdot slot is never read
  }
  for (int pos = tid; pos < n * bp; pos += nt) {
    const int m = pos / bp, t = pos - m * bp, i = m + t;
    Lf[pos] = i < n ? w1s * sy.Mb[(size_t)i * W2 + (bw - t)] : 0.0;
    if (vel) Ct[pos] = i < n ? ct_entry(sy, q, qd, pos) : 0.0;
  }
  __syncthreads();
  band_ldlt(Lf, n, bw, st);
  band_solve(Lf, n, bw, a, red);
  // (w1^2 M) Aw_0 = -(D + C_t) u0 - 2 w1 M a0
  for (int i = tid; i < n; i += nt) {
    double v = 0.0;
    for (int t = 0; t < W2; ++t) {
      const int j = i - bw + t;
      if (j < 0 || j >= n) continue;
      const double Dij = sy.Db[(size_t)i * W2 + t] + (vel ? ct_band(Ct, bp, i, j) : 0.0);
      v -= Dij * u[j] + 2.0 * w1 * sy.Mb[(size_t)i * W2 + t] * a[j];
    }
    x[i] = v;
  }
  __syncthreads();
  band_solve(Lf, n, bw, x, red);
  for (int i = tid; i < n; i += nt) {
    Qw[i] = 0.0;
    Uw[i] = 0.0;
    Aw[i] = x[i];
  }
  __syncthreads();

  for (int k = 0; k < P.S1; ++k) {
    for (int i = tid; i < n; i += nt) {
      qn[i] = qhist[((size_t)(k + 1) * n + i) * ldw + w];
      // qdot of the step's end state, for C_t: u_{k+1} follows from q_{k+1} (Newmark relations)
      if (vel) qd[i] = w1 * (P.c2 * (qn[i] - q[i]) - P.d1 * u[i] - P.d2 * a[i]);
    }
    __syncthreads();
    if (vel) {
      for (int pos = tid; pos < n * bp; pos += nt) {
        const int m = pos / bp, i = m + (pos - m * bp);
        Ct[pos] = i < n ? ct_entry(sy, qn, qd, pos) : 0.0;
      }
      __syncthreads();
    }
    for (int i = tid; i < n; i += nt) {
      double v = 0.0;
      for (int t = 0; t < W2; ++t) {
        const int j = i - bw + t;
        if (j < 0 || j >= n) continue;
        // the velocity-dependent forces linearise into the damping D + C_t
        const double Mij = sy.Mb[(size_t)i * W2 + t];
        const double Dij = sy.Db[(size_t)i * W2 + t] + (vel ? ct_band(Ct, bp, i, j) : 0.0);
        v += w1s * Mij * (P.c0 * Qw[j] + P.c1 * Uw[j] + P.c3 * Aw[j]) + w1 * Dij * (P.c2 * Qw[j] + P.d1 * Uw[j] + P.d2 * Aw[j]);
        v += -(2.0 * w1 * P.c0 * Mij + P.c2 * Dij) * qn[j] +
             2.0 * w1 * Mij * (P.c0 * q[j] + P.c1 * u[j] + P.c3 * a[j]) + Dij * (P.c2 * q[j] + P.d1 * u[j] + P.d2 * a[j]);
      }
      x[i] = v;
    }
    for (int pos = tid; pos < n * bp; pos += nt) {
      const int m = pos / bp, t = pos - m * bp, i = m + t;
      double v = 0.0;
      if (i < n) {
        const size_t e = (size_t)i * W2 + (bw - t);
        v = w1s * P.c0 * sy.Mb[e] + w1 * P.c2 * sy.Db[e] + sy.Kb[e] + kt_entry(sy, qn, vel ? qd : qn, pos);
        if (vel) v += w1 * P.c2 * Ct[pos];
      }
      Lf[pos] = v;
    }
    __syncthreads();
    band_ldlt(Lf, n, bw, st);
    band_solve(Lf, n, bw, x, red);
    for (int i = tid; i < n; i += nt) {
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
    __syncthreads();
  }
  bool nan = false;
  for (int i = tid; i < n; i += nt) {
    dzT[(size_t)i * ldw + w] = Qw[i];
    dzT[(size_t)(n + i) * ldw + w] = Uw[i];
    if (!isfinite(Qw[i]) || !isfinite(Uw[i])) nan = true;
  }
  if (nan) atomicOr(&st->flags, (int)DEV_NAN);
}

// ------------------------------------------------------------------------ DFT, rotation, residual
// R = (I (x) R(rho)) (I (x) Gamma^-1) zbar(2 pi) - Z(0)   (Eqs. 15, 16, 21)
__global__ void k_dft_residual(const double *__restrict__ zT, int ldw, const double *__restrict__ Gi,
                               const double *__restrict__ rot, const double *__restrict__ Z0, int n,
                               int U, int L, int St, int B, double *__restrict__ R) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = B * 2 * n * (L + 1);
  if (idx >= total) return;
  const int l = idx % (L + 1);
  const int bi = idx / (L + 1);
  const int i = bi % (2 * n), b = bi / (2 * n);
  const double *z = zT + (size_t)i * ldw + (size_t)b * St;
  const double *z0 = Z0 + ((size_t)b * 2 * n + i) * U;
  double *r = R + ((size_t)b * 2 * n + i) * U;
  if (l == L) {
    double v = 0.0;
    for (int s = 0; s < St; ++s) v += Gi[s] * z[s];
    r[0] = v - z0[0];
    return;
  }
  const double *gc = Gi + (size_t)(2 * l + 1) * St;
  const double *gs = Gi + (size_t)(2 * l + 2) * St;
  double cc = 0.0, ss = 0.0;
  for (int s = 0; s < St; ++s) {
    cc += gc[s] * z[s];
    ss += gs[s] * z[s];
  }
  const double al = rot[(size_t)b * (L > 0 ? L : 1) + l];
  const double ca = cos(al), sa = sin(al);
  r[2 * l + 1] = ca * cc - sa * ss - z0[2 * l + 1];
  r[2 * l + 2] = sa * cc + ca * ss - z0[2 * l + 2];
}

__global__ void k_sumsq(const double *__restrict__ R, size_t len, double *__restrict__ out) {
  __shared__ double red[16];
  const double *r = R + (size_t)blockIdx.x * len;
  double v = 0.0;
  for (size_t i = threadIdx.x; i < len; i += blockDim.x) v += r[i] * r[i];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    out[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------------ Jacobian (Eq. 22)
// P[s][l][m] = (R Gamma^-1)[l][s] Gamma[s][m]
__global__ void k_jac_P(const double *__restrict__ Gi, const double *__restrict__ G,
                        const double *__restrict__ rot, int U, int L, int St,
                        double *__restrict__ Pm) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)St * U * U;
  if (idx >= total) return;
  const int m = idx % U;
  const int l = (idx / U) % U;
  const int s = idx / ((size_t)U * U);
  double a;
  if (l == 0) {
    a = Gi[s];
  } else {
    const int pr = (l - 1) / 2;
    const double al = rot[pr], ca = cos(al), sa = sin(al);
    const double gc = Gi[(size_t)(2 * pr + 1) * St + s], gs = Gi[(size_t)(2 * pr + 2) * St + s];
    a = (l & 1) ? (ca * gc - sa * gs) : (sa * gc + ca * gs);
  }
  Pm[idx] = a * G[(size_t)s * U + m];
}

// J[(i,l),(j,m)] = sum_s Phi_s[i][j] P[s][l][m] - delta: GEMM over s with
// 64 (ij) x 64 (lm) tiles, 4 x 4 outputs per thread.
__global__ __launch_bounds__(256) void k_jac_gemm(const double *__restrict__ Phi,
                                                  const double *__restrict__ Pm, int n2, int U,
                                                  int St, double *__restrict__ J, size_t ldJ) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const size_t NIJ = (size_t)n2 * n2;
  const int NLM = U * U;
  const size_t ij0 = (size_t)blockIdx.x * 64;
  const int lm0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int s0 = 0; s0 < St; s0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int ks = e / 64, col = e % 64;
      const int s = s0 + ks;
      const size_t ij = ij0 + col;
      As[ks][col] = (s < St && ij < NIJ) ? Phi[(size_t)s * NIJ + ij] : 0.0;
      const int lm = lm0 + col;
      Bs[ks][col] = (s < St && lm < NLM) ? Pm[(size_t)s * NLM + lm] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[ks][ty * 4 + a];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[ks][tx * 4 + c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] += av[a] * bv[c];
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const size_t ij = ij0 + ty * 4 + a;
    if (ij >= NIJ) continue;
    const int i = (int)(ij / n2), j = (int)(ij % n2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int lm = lm0 + tx * 4 + c;
      if (lm >= NLM) continue;
      const int l = lm / U, m = lm % U;
      const size_t row = (size_t)i * U + l, col = (size_t)j * U + m;
      J[row * ldJ + col] = acc[a][c] - ((row == col) ? 1.0 : 0.0);
    }
  }
}

SysDev sysdev(const fse_ctx *ctx) {
  return SysDev{ctx->Mb,     ctx->Db,     ctx->Kb,     ctx->F,      ctx->f2_ptr, ctx->f2_jk, ctx->f2_v,
                ctx->f3_ptr, ctx->f3_jkl, ctx->f3_v,   ctx->kt_ptr, ctx->kt_idx, ctx->kt_c,
                ctx->has_vel ? ctx->ct_ptr : nullptr,   ctx->ct_idx, ctx->ct_c,
                ctx->ncon ? ctx->cn_ptr : nullptr,      ctx->cn_v,   ctx->bw,     ctx->n};
}

TrajParams params(const fse_ctx *ctx, int B) {
  TrajParams P;
  P.n = ctx->n;
  P.bw = ctx->bw;
  P.S1 = ctx->seg_steps > 0 ? ctx->seg_steps : ctx->S1;
  P.phib = ctx->seg_phase;
  P.e = ctx->e;
  P.d = ctx->d;
  P.St = ctx->St;
  P.W = B * ctx->St;
  P.maxit = ctx->maxit;
  P.tol = ctx->tol;
  newmark_coefficients(ctx, P);
  return P;
}

constexpr size_t kLdsLimit = 64 * 1024;

}  // namespace

fse_status reset_status(fse_ctx *ctx) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, ctx->stream, ctx->status_d, INT_MAX);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_idft(fse_ctx *ctx, int B, const double *Z0) {
  const int W = B * ctx->St;
  dim3 grid((W + 127) / 128, 2 * ctx->n);
  hipLaunchKernelGGL(k_idft, grid, dim3(128), 0, ctx->stream, Z0, ctx->G_d, ctx->n, ctx->U, ctx->St, W,
                     ctx->Wmax, ctx->qhist, ctx->u0);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

// Global scratch of the state and omega_1-sensitivity kernels when their per-trajectory
// working set exceeds LDS; the two kernels have different strides, so the buffer grows to the
// larger request (the stream is drained before a reallocation).
fse_status ensure_state_scr(fse_ctx *ctx, size_t elems) {
  if (ctx->state_scr_elems >= elems) return FSE_OK;
  if (ctx->state_scr) {
    FSE_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->state_scr);
  }
  ctx->state_scr = nullptr;
  ctx->state_scr_elems = 0;
  if (hipMalloc((void **)&ctx->state_scr, sizeof(double) * elems) != hipSuccess) {
    ctx->err = "hipMalloc failed for the state scratch";
    return FSE_E_NOMEM;
  }
  ctx->state_scr_elems = elems;
  return FSE_OK;
}

fse_status launch_state(fse_ctx *ctx, int B) {
  const TrajParams P = params(ctx, B);
  const size_t elems = (size_t)ctx->n * (ctx->bw + 1) + 9 * (size_t)ctx->n + 80;
  double *uh = ctx->has_vel ? ctx->uhist : nullptr;
  const size_t bytes = elems * sizeof(double);
  // reset the status word; the first failing step starts at "none"
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, ctx->stream, ctx->status_d, INT_MAX);
  const int threads = ctx->bw > 24 ? 256 : 64;
  if (bytes <= kLdsLimit) {
    hipLaunchKernelGGL(k_state<true>, dim3(P.W), dim3(threads), bytes, ctx->stream, P, sysdev(ctx),
                       ctx->omega_d, ctx->sidx_d, ctx->Sdim_d, ctx->qhist, uh, ctx->u0, ctx->zTw,
                       ctx->Wmax, nullptr, ctx->status_d);
  } else {
    FSE_TRY(ensure_state_scr(ctx, elems * ctx->Wmax));
    hipLaunchKernelGGL(k_state<false>, dim3(P.W), dim3(threads), 0, ctx->stream, P, sysdev(ctx),
                       ctx->omega_d, ctx->sidx_d, ctx->Sdim_d, ctx->qhist, uh, ctx->u0, ctx->zTw,
                       ctx->Wmax, ctx->state_scr, ctx->status_d);
  }
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_sens(fse_ctx *ctx, int B, double *PhiQU) {
  const TrajParams P = params(ctx, B);
  const size_t n = ctx->n, n2 = 2 * n;
  if (!ctx->PhiA) {
    if (hipMalloc((void **)&ctx->PhiA, sizeof(double) * ctx->Wmax * n * n2) != hipSuccess ||
        hipMalloc((void **)&ctx->sens_scr, sizeof(double) * ctx->Wmax * n * n2) != hipSuccess) {
      ctx->err = "hipMalloc failed for the sensitivity buffers";
      return FSE_E_NOMEM;
    }
  }
  const int C = ctx->sens_cols;
  const int nblk = (int)((n2 + C - 1) / C);
  const size_t elems = 3 * n * (ctx->bw + 1) + 2 * n + 8;
  const double *uh = ctx->has_vel ? ctx->uhist : nullptr;
  const size_t bytes = elems * sizeof(double);
  dim3 grid(nblk, P.W);
  if (bytes <= kLdsLimit) {
    hipLaunchKernelGGL(k_sens<true>, grid, dim3(C), bytes, ctx->stream, P, sysdev(ctx), ctx->omega_d,
                       ctx->qhist, uh, ctx->Wmax, PhiQU, ctx->PhiA, ctx->sens_scr, nullptr, ctx->status_d);
  } else {
    const size_t need = elems * nblk * (size_t)ctx->Wmax;
    if (ctx->sens_gscr_elems < need) {
      if (ctx->sens_gscr) (void)hipFree(ctx->sens_gscr);
      ctx->sens_gscr = nullptr;
      ctx->sens_gscr_elems = 0;
      if (hipMalloc((void **)&ctx->sens_gscr, sizeof(double) * need) != hipSuccess) {
        ctx->err = "hipMalloc failed for the sensitivity factor scratch";
        return FSE_E_NOMEM;
      }
      ctx->sens_gscr_elems = need;
    }
    hipLaunchKernelGGL(k_sens<false>, grid, dim3(C), 0, ctx->stream, P, sysdev(ctx), ctx->omega_d,
                       ctx->qhist, uh, ctx->Wmax, PhiQU, ctx->PhiA, ctx->sens_scr, ctx->sens_gscr,
                       ctx->status_d);
  }
  ctx->last_sens_launches = 1;
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_dft_residual(fse_ctx *ctx, int B, const double *Z0, double *R) {
  return launch_dft(ctx, B, ctx->zTw, Z0, R);
}

fse_status launch_dft(fse_ctx *ctx, int B, const double *zT, const double *Z0, double *R, const double *rot) {
  const int total = B * 2 * ctx->n * (ctx->L + 1);
  hipLaunchKernelGGL(k_dft_residual, dim3((total + 255) / 256), dim3(256), 0, ctx->stream, zT,
                     ctx->Wmax, ctx->Gi_d, rot ? rot : ctx->rot_d, Z0, ctx->n, ctx->U, ctx->L, ctx->St, B, R);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_norms(fse_ctx *ctx, int B, const double *R, double *out_host) {
  hipLaunchKernelGGL(k_sumsq, dim3(B), dim3(256), 0, ctx->stream, R, (size_t)2 * ctx->n * ctx->U,
                     ctx->norm_d);
  FSE_HIP(hipGetLastError());
  std::vector<double> h(B);
  FSE_HIP(hipMemcpyAsync(h.data(), ctx->norm_d, sizeof(double) * B, hipMemcpyDeviceToHost, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  for (int b = 0; b < B; ++b) out_host[b] = std::sqrt(h[b]);
  return FSE_OK;
}

// Border of the Newton matrix for the unknown base frequencies omega_f, f = e..d-1
// (0-based): column N + u holds dR/d omega_f (Eqs. 23-24, rotation term only, since the
// forcing does not depend on a response frequency), computed from (R + Z0) = R(rho) Z(2 pi);
// row N + u holds the phase row [(I (x) nabla_f) Z0]^T of Eq. (18); the corner is zero.
__global__ void k_border(double *__restrict__ Jb, size_t ldJ, int N, int nu, const double *__restrict__ R,
                         const double *__restrict__ Z0, const int32_t *__restrict__ ktable, int L, int dm1,
                         int e, double two_pi_over_w1, int U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nu) return;
  const int u = idx / N, r = idx - u * N;
  const int a = r % U, base = r - a;
  const int fcol = e + u - 1;  // harmonic-table column of frequency e + u (0-based)
  double dr = 0.0, pr = 0.0;
  if (a > 0) {
    const int l = (a - 1) / 2;
    const double k = (double)ktable[(size_t)l * dm1 + fcol];
    if (a & 1) {  // cos coefficient 2l+1
      dr = -two_pi_over_w1 * k * (R[base + a + 1] + Z0[base + a + 1]);
      pr = k * Z0[base + a + 1];
    } else {      // sin coefficient 2l+2
      dr = two_pi_over_w1 * k * (R[base + a - 1] + Z0[base + a - 1]);
      pr = -k * Z0[base + a - 1];
    }
  }
  Jb[(size_t)r * ldJ + N + u] = dr;
  Jb[(size_t)(N + u) * ldJ + r] = pr;
  if (r < nu) Jb[(size_t)(N + u) * ldJ + N + r] = 0.0;
}

fse_status launch_border(fse_ctx *ctx, double *Jb, size_t ldJ, const double *R, const double *Z0,
                         double omega1) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  if (nu <= 0) return FSE_OK;
  hipLaunchKernelGGL(k_border, dim3((N * nu + 255) / 256), dim3(256), 0, ctx->stream, Jb, ldJ, N, nu, R, Z0,
                     ctx->ktable_d, ctx->L, ctx->d - 1, ctx->e, 2.0 * M_PI / omega1, ctx->U);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

// dR/d omega_f for the unknown base frequencies alone: out [N][nu] (same terms as k_border).
__global__ void k_dRdw(double *__restrict__ out, int N, int nu, const double *__restrict__ R,
                       const double *__restrict__ Z0, const int32_t *__restrict__ ktable, int dm1, int e,
                       double two_pi_over_w1, int U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nu) return;
  const int u = idx / N, r = idx - u * N;
  const int a = r % U, base = r - a;
  double dr = 0.0;
  if (a > 0) {
    const int l = (a - 1) / 2;
    const double k = (double)ktable[(size_t)l * dm1 + e + u - 1];
    dr = (a & 1) ? -two_pi_over_w1 * k * (R[base + a + 1] + Z0[base + a + 1])
                 : two_pi_over_w1 * k * (R[base + a - 1] + Z0[base + a - 1]);
  }
  out[(size_t)r * nu + u] = dr;
}

fse_status launch_dRdw(fse_ctx *ctx, double *out, const double *R, const double *Z0, double omega1) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  if (nu <= 0) return FSE_OK;
  hipLaunchKernelGGL(k_dRdw, dim3((N * nu + 255) / 256), dim3(256), 0, ctx->stream, out, N, nu, R, Z0,
                     ctx->ktable_d, ctx->d - 1, ctx->e, 2.0 * M_PI / omega1, ctx->U);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

// dR/dp -= sum_u rho_u dR/d omega_u (u = e..d-1): with omega_u held while omega_1 = p moves,
// rho_u = omega_u / omega_1 changes by -rho_u / omega_1 per unit p; the rotation term of
// dR/d omega_u (Eqs. 23-24, as in k_dRdw) is taken from R + Z0 = R(rho) Z(2 pi).
struct RhoU {
  double v[8];
};

__global__ void k_dRdp_rot(double *__restrict__ dRdp, int N, int nu, const double *__restrict__ R,
                           const double *__restrict__ Z0, const int32_t *__restrict__ ktable, int dm1,
                           int e, double two_pi_over_w1, int U, RhoU rho) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int a = r % U, base = r - a;
  if (a == 0) return;
  const int l = (a - 1) / 2;
  double acc = 0.0;
  for (int u = 0; u < nu; ++u) {
    const double k = (double)ktable[(size_t)l * dm1 + e + u - 1];
    const double dr = (a & 1) ? -two_pi_over_w1 * k * (R[base + a + 1] + Z0[base + a + 1])
                              : two_pi_over_w1 * k * (R[base + a - 1] + Z0[base + a - 1]);
    acc += rho.v[u] * dr;
  }
  dRdp[r] -= acc;
}

// Column N + nu of the arclength matrix: dR/dp in rows 0..N-1, zero in the phase rows.
__global__ void k_set_pcol(double *__restrict__ A, size_t ldA, int N, int nu, const double *__restrict__ col) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N + nu) return;
  A[(size_t)r * ldA + N + nu] = r < N ? col[r] : 0.0;
}

fse_status launch_wsens(fse_ctx *ctx, int B, double *dzT) {
  const fse_status fs = ctx->wsens_generic ? FSE_E_UNSUPPORTED : launch_wsens_fused(ctx, B, dzT);
  if (fs != FSE_E_UNSUPPORTED) return fs;
  const TrajParams P = params(ctx, B);
  const size_t nb = (size_t)ctx->n * (ctx->bw + 1);
  const size_t elems = nb + 8 * (size_t)ctx->n + 80 + (ctx->has_vel ? nb + ctx->n : 0);
  const size_t bytes = elems * sizeof(double);
  const int threads = ctx->bw > 24 ? 256 : 64;
  if (bytes <= kLdsLimit) {
    hipLaunchKernelGGL(k_wsens<true>, dim3(P.W), dim3(threads), bytes, ctx->stream, P, sysdev(ctx),
                       ctx->omega_d, ctx->sidx_d, ctx->Sdim_d, ctx->qhist, ctx->u0, ctx->Wmax, dzT, nullptr,
                       ctx->status_d);
  } else {
    FSE_TRY(ensure_state_scr(ctx, elems * ctx->Wmax));
    hipLaunchKernelGGL(k_wsens<false>, dim3(P.W), dim3(threads), 0, ctx->stream, P, sysdev(ctx),
                       ctx->omega_d, ctx->sidx_d, ctx->Sdim_d, ctx->qhist, ctx->u0, ctx->Wmax, dzT,
                       ctx->state_scr, ctx->status_d);
  }
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_dRdp_rot(fse_ctx *ctx, int B, const double *omega, const double *R, const double *Z0,
                           double *dRdp) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  if (nu <= 0) return FSE_OK;
  if (nu > 8) {
    ctx->err = "at most 8 unknown base frequencies";
    return FSE_E_UNSUPPORTED;
  }
  for (int b = 0; b < B; ++b) {
    const double *om = omega + (size_t)b * ctx->d;
    RhoU rho{};
    for (int u = 0; u < nu; ++u) rho.v[u] = om[ctx->e + u] / om[0];
    hipLaunchKernelGGL(k_dRdp_rot, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, dRdp + (size_t)b * N, N,
                       nu, R + (size_t)b * N, Z0 + (size_t)b * N, ctx->ktable_d, ctx->d - 1, ctx->e,
                       2.0 * M_PI / om[0], ctx->U, rho);
  }
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_set_pcol(fse_ctx *ctx, double *A, size_t ldA, const double *col) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  hipLaunchKernelGGL(k_set_pcol, dim3((N + nu + 255) / 256), dim3(256), 0, ctx->stream, A, ldA, N, nu, col);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_norm(fse_ctx *ctx, const double *x, size_t len, double *out_host) {
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, ctx->stream, x, len, ctx->norm_d);
  FSE_HIP(hipGetLastError());
  double h = 0.0;
  FSE_HIP(hipMemcpyAsync(&h, ctx->norm_d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  *out_host = std::sqrt(h);
  return FSE_OK;
}

fse_status launch_jacobian(fse_ctx *ctx, int B, const double *PhiQU, double *J, size_t ldJ) {
  const int U = ctx->U, St = ctx->St, n2 = 2 * ctx->n;
  const size_t Pn = (size_t)St * U * U;
  if (!ctx->jacP && hipMalloc((void **)&ctx->jacP, sizeof(double) * Pn) != hipSuccess) {
    ctx->err = "hipMalloc failed for the Jacobian factor";
    return FSE_E_NOMEM;
  }
  double *Pm = ctx->jacP;
  const size_t N = (size_t)n2 * U;
  for (int b = 0; b < B; ++b) {
    hipLaunchKernelGGL(k_jac_P, dim3((unsigned)((Pn + 255) / 256)), dim3(256), 0, ctx->stream, ctx->Gi_d,
                       ctx->G_d, ctx->rot_d + (size_t)b * (ctx->L > 0 ? ctx->L : 1), U, ctx->L, St, Pm);
    const size_t NIJ = (size_t)n2 * n2;
    dim3 grid((unsigned)((NIJ + 63) / 64), (unsigned)((U * U + 63) / 64));
    hipLaunchKernelGGL(k_jac_gemm, grid, dim3(256), 0, ctx->stream,
                       PhiQU + (size_t)b * St * NIJ, Pm, n2, U, St, J + (size_t)b * N * ldJ, ldJ);
  }
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}
