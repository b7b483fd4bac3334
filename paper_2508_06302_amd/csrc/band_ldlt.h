// Banded LDL^T kernels-in-a-lane shared by the trajectory kernels (App. E, Eqs. E6-E9):
// the tangent T = S + K_t(q) assembled in LDS from the sparse polynomial forces, its
// factorisation and solves by one lane with register windows.  Every translation unit that
// includes this header gets its own copies (anonymous namespace).
//
// Padded LDL^T storage [n+BW][BW+1]: entry (j + r, j) at [BW + j][r], [BW + j][0] = 1 / d_j;
// the BW leading rows are zero so sweeps need no guards.  Full rows [n][2BW+1]: entry (i, j)
// at [i][j - i + BW].
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace {

// LDS-qualified element type: the serial factor and solve routines below are not always
// inlined, and a generic pointer argument would make every access a flat instruction.
typedef __attribute__((address_space(3))) double lds_double;

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

// Polynomial forces: row pointers, packed indices and values.  TensLds points to LDS (the
// staged copy of the fused kernel), TensGlb to global memory; the address space is part of the
// type so that no access goes through a generic pointer.
typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(1))) const int glb_int;
typedef __attribute__((address_space(1))) const uint32_t glb_u32;
typedef __attribute__((address_space(1))) const double glb_double;

template <typename I, typename W, typename D>
struct TensT {
  const I *p2, *p3;
  const W *i2, *i3;
  const D *v2, *v3;
};
using TensLds = TensT<lds_int, lds_u32, lds_double>;
using TensGlb = TensT<glb_int, glb_u32, glb_double>;

// f_nl(q)_i = sum t2 q_j q_k + sum t3 q_j q_k q_l over row i (four partial sums)
template <typename TL>
__device__ inline double fnl_row(const TL &t, const double *q_, int i) {
  const lds_double *q = (const lds_double *)q_;  // q is in LDS for every caller
  double f[4] = {0.0, 0.0, 0.0, 0.0};
  const int a0 = t.p2[i], a1 = t.p2[i + 1];
  int p = a0;
  for (; p + 3 < a1; p += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t x = t.i2[p + u];
      f[u] += t.v2[p + u] * q[x & 0xffff] * q[x >> 16];
    }
  }
  for (; p < a1; ++p) {
    const uint32_t x = t.i2[p];
    f[0] += t.v2[p] * q[x & 0xffff] * q[x >> 16];
  }
  const int b0 = t.p3[i], b1 = t.p3[i + 1];
  p = b0;
  for (; p + 3 < b1; p += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t x = t.i3[2 * (p + u)], xl = t.i3[2 * (p + u) + 1];
      f[u] += t.v3[p + u] * q[x & 0xffff] * q[x >> 16] * q[xl];
    }
  }
  for (; p < b1; ++p) {
    const uint32_t x = t.i3[2 * p], xl = t.i3[2 * p + 1];
    f[1] += t.v3[p] * q[x & 0xffff] * q[x >> 16] * q[xl];
  }
  return (f[0] + f[1]) + (f[2] + f[3]);
}

// Lower band of T = S + K_t(q) into F (padded column storage), lanes of one wave over
// rows: the lane of row i owns the entries (i, i - r), so no two lanes write the same
// word.  K_t(i, m) = d f_i / d q_m collects the terms of row i whose index set holds m
// (entries with m > i are the transposes of lower entries of a symmetric tangent).
template <int BW, bool BandLds = false, typename TL>
__device__ void assemble_T(const TL t, int n, const double *__restrict__ Sp_, const double *q_,
                           double *Fp, int lane) {
  constexpr int bp = BW + 1, W2 = 2 * BW + 1;
  // q and the factor are in LDS; the band S is in global memory, or in LDS (BandLds)
  typedef __attribute__((address_space(1))) const double gcdouble;
  const lds_double *q = (const lds_double *)q_;
  lds_double *F = (lds_double *)Fp + BW * bp;
  for (int i = lane; i < n; i += 64) {
#pragma unroll
    for (int r = 0; r <= BW; ++r) {
      const int m = i - r;
      if (m >= 0) {
        const size_t e = (size_t)i * W2 + (BW - r);
        F[m * bp + r] = BandLds ? ((const lds_double *)Sp_)[e] : ((gcdouble *)Sp_)[e];
      }
    }
    for (int p = t.p2[i]; p < t.p2[i + 1]; ++p) {
      const uint32_t x = t.i2[p];
      const int j = x & 0xffff, k = x >> 16;
      const double v = t.v2[p];
      if (j <= i) F[j * bp + (i - j)] += v * q[k];
      if (k <= i) F[k * bp + (i - k)] += v * q[j];
    }
    for (int p = t.p3[i]; p < t.p3[i + 1]; ++p) {
      const uint32_t x = t.i3[2 * p];
      const int j = x & 0xffff, k = x >> 16, l = t.i3[2 * p + 1];
      const double v = t.v3[p];
      if (j <= i) F[j * bp + (i - j)] += v * q[k] * q[l];
      if (k <= i) F[k * bp + (i - k)] += v * q[j] * q[l];
      if (l <= i) F[l * bp + (i - l)] += v * q[j] * q[k];
    }
  }
}

// In-place banded LDL^T by one lane with a register window (padded storage, see
// file header).  Returns false on a zero or non-finite pivot.
template <int BW>
__device__ bool ldlt_serial_shift(lds_double *Fp, int n) {
  constexpr int bp = BW + 1;
  lds_double *F = Fp + BW * bp;
  double Wn[BW + 1][BW + 1];
#pragma unroll
  for (int r = 0; r <= BW; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) Wn[r][c] = (r < n) ? F[c * bp + (r - c)] : 0.0;
  bool ok = true;
  for (int j = 0; j < n; ++j) {
    const double d = Wn[0][0];
    ok = ok && (d != 0.0) && isfinite(d);
    // reciprocal: hardware estimate refined by one Newton step (relative error ~1 ulp)
    double inv = __builtin_amdgcn_rcp(d);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    double l[BW + 1];
#pragma unroll
    for (int r = 1; r <= BW; ++r) l[r] = Wn[r][0] * inv;
    F[j * bp] = inv;
#pragma unroll
    for (int r = 1; r <= BW; ++r) F[j * bp + r] = (j + r < n) ? l[r] : 0.0;
#pragma unroll
    for (int r = 1; r <= BW; ++r)
#pragma unroll
      for (int c = 1; c <= r; ++c) Wn[r][c] -= Wn[r][0] * l[c];
#pragma unroll
    for (int r = 0; r < BW; ++r)
#pragma unroll
      for (int c = 0; c <= r; ++c) Wn[r][c] = Wn[r + 1][c + 1];
    const bool in = j + 1 + BW < n;
#pragma unroll
    for (int c = 0; c <= BW; ++c) Wn[BW][c] = in ? F[(j + 1 + c) * bp + (BW - c)] : 0.0;
  }
  return ok;
}

// Solve (L D L^T) x = x in place by one lane.  The coefficients of the next row
// are loaded while the current row is reduced, and the term with the most recent
// unknown is applied last, so each row adds one dependent FMA to the critical path.
template <int BW>
__device__ void ldlt_solve_shift(const lds_double *Fp, int n, lds_double *x) {
  constexpr int bp = BW + 1;
  const lds_double *F = Fp + BW * bp;
  double yw[BW], cf[BW + 1], cn[BW + 1];
#pragma unroll
  for (int t = 0; t < BW; ++t) yw[t] = 0.0;
#pragma unroll
  for (int t = 1; t <= BW; ++t) cf[t] = F[(0 - t) * bp + t];
  double xn = x[0];
  for (int i = 0; i < n; ++i) {
    const double xi = xn;
    const int i1 = i + 1 < n ? i + 1 : i;
#pragma unroll
    for (int t = 1; t <= BW; ++t) cn[t] = F[(i1 - t) * bp + t];
    xn = x[i1];
    // older terms in two independent partial sums, off the critical path
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int t = BW; t >= 2; --t) {
      if ((t & 1) == 0)
        s0 += cf[t] * yw[t - 1];
      else
        s1 += cf[t] * yw[t - 1];
    }
    const double acc = (xi - (s0 + s1)) - cf[1] * yw[0];
#pragma unroll
    for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
    yw[0] = acc;
    x[i] = acc;
#pragma unroll
    for (int t = 1; t <= BW; ++t) cf[t] = cn[t];
  }
#pragma unroll
  for (int t = 0; t < BW; ++t) yw[t] = 0.0;
#pragma unroll
  for (int t = 0; t <= BW; ++t) cf[t] = F[(n - 1) * bp + t];
  xn = x[n - 1];
  for (int i = n - 1; i >= 0; --i) {
    const double xi = xn;
    const int i1 = i > 0 ? i - 1 : 0;
#pragma unroll
    for (int t = 0; t <= BW; ++t) cn[t] = F[i1 * bp + t];
    xn = x[i1];
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int t = BW; t >= 2; --t) {
      if ((t & 1) == 0)
        s0 += cf[t] * yw[t - 1];
      else
        s1 += cf[t] * yw[t - 1];
    }
    const double acc = (xi * cf[0] - (s0 + s1)) - cf[1] * yw[0];
#pragma unroll
    for (int t = BW - 1; t >= 1; --t) yw[t] = yw[t - 1];
    yw[0] = acc;
    x[i] = acc;
#pragma unroll
    for (int t = 0; t <= BW; ++t) cf[t] = cn[t];
  }
}

// Register-ring variants for half bandwidths up to 6 (P = BW + 1 slots).
// Factorisation: entry A(R, C) of the active window lives in G[R % P][C % P]; with the
// column loop unrolled by P every slot index is a compile-time constant, so the window
// never moves between registers.  The row entering the window after column j (row
// j + P) is loaded at the end of column j, one column ahead of its first use.
template <int BW>
__device__ bool ldlt_serial_ring(lds_double *Fp, int n) {
  constexpr int P = BW + 1, bp = BW + 1;
  lds_double *F = Fp + BW * bp;
  double G[P][P];
#pragma unroll
  for (int r = 0; r < P; ++r)
#pragma unroll
    for (int c = 0; c < P; ++c) G[r][c] = (c <= r && r < n) ? F[c * bp + (r - c)] : 0.0;
  bool ok = true;
  for (int j0 = 0; j0 < n; j0 += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int j = j0 + u;
      if (j >= n) break;
      const double d = G[u][u];
      ok = ok && (d != 0.0) && isfinite(d);
      // reciprocal: hardware estimate refined by one Newton step
      double inv = __builtin_amdgcn_rcp(d);
      inv = fma(inv, fma(-d, inv, 1.0), inv);
      double l[P];
#pragma unroll
      for (int t = 1; t <= BW; ++t) l[t] = G[(u + t) % P][u] * inv;
      F[j * bp] = inv;
#pragma unroll
      for (int t = 1; t <= BW; ++t) F[j * bp + t] = l[t];
#pragma unroll
      for (int r = 1; r <= BW; ++r)
#pragma unroll
        for (int c = 1; c <= r; ++c) G[(u + r) % P][(u + c) % P] -= G[(u + r) % P][u] * l[c];
      // row R = j + P enters slot u: A(R, C) for C = j + 1 .. j + P
      const int R = j + P;
      const bool in = R < n;
#pragma unroll
      for (int c = 0; c <= BW; ++c) {
        const int C = j + 1 + c;
        G[u][(u + 1 + c) % P] = in ? F[C * bp + (R - C)] : 0.0;
      }
    }
  }
  return ok;
}

// Solve (L D L^T) x = x in place by one lane; step k of each sweep keeps its result in
// slot k % P of a register ring and the coefficients of step k + P are loaded when step
// k retires, P steps before they are needed.  The term of the newest unknown is
// applied last, so each row adds one dependent FMA to the critical path.
template <int BW>
__device__ void ldlt_solve_ring(const lds_double *Fp, int n, lds_double *x) {
  constexpr int P = BW + 1, bp = BW + 1;
  const lds_double *F = Fp + BW * bp;
  double y[P], cf[P][P], xv[P];
  // forward: row i = k, coefficients L(i, i - t) = F[(i - t) bp + t]
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int ir = u < n ? u : n - 1;
    y[u] = 0.0;
    xv[u] = x[ir];
#pragma unroll
    for (int t = 1; t <= BW; ++t) cf[u][t] = F[(ir - t) * bp + t];
  }
  for (int k0 = 0; k0 < n; k0 += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int i = k0 + u;
      if (i >= n) break;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int t = BW; t >= 2; --t) {
        if ((t & 1) == 0)
          s0 += cf[u][t] * y[(u - t + P) % P];
        else
          s1 += cf[u][t] * y[(u - t + P) % P];
      }
      const double acc = (xv[u] - (s0 + s1)) - cf[u][1] * y[(u - 1 + P) % P];
      y[u] = acc;
      x[i] = acc;
      const int ir = i + P < n ? i + P : n - 1;
      xv[u] = x[ir];
#pragma unroll
      for (int t = 1; t <= BW; ++t) cf[u][t] = F[(ir - t) * bp + t];
    }
  }
  // backward: row i = n - 1 - k, coefficients D^-1 = F[i bp], L(i + t, i) = F[i bp + t]
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int ir = n - 1 - u >= 0 ? n - 1 - u : 0;
    y[u] = 0.0;
    xv[u] = x[ir];
#pragma unroll
    for (int t = 0; t <= BW; ++t) cf[u][t] = F[ir * bp + t];
  }
  for (int k0 = 0; k0 < n; k0 += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int k = k0 + u;
      if (k >= n) break;
      const int i = n - 1 - k;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int t = BW; t >= 2; --t) {
        if ((t & 1) == 0)
          s0 += cf[u][t] * y[(u - t + P) % P];
        else
          s1 += cf[u][t] * y[(u - t + P) % P];
      }
      const double acc = (xv[u] * cf[u][0] - (s0 + s1)) - cf[u][1] * y[(u - 1 + P) % P];
      y[u] = acc;
      x[i] = acc;
      const int ir = i - P >= 0 ? i - P : 0;
      xv[u] = x[ir];
#pragma unroll
      for (int t = 0; t <= BW; ++t) cf[u][t] = F[ir * bp + t];
    }
  }
}

// Chord factor in FP32 (half bandwidths up to 6).  The chord matrix of the per-step
// Newton iteration (Eq. E6) only has to approximate the tangent: the residual stays FP64,
// so a factor rounded to FP32 changes the contraction of the iteration, not its fixed
// point.  Storage: rows of 8 floats, [j][0] = 1 / d_j, [j][t] = L(j + t, j) for
// t = 1..BW, the rest zero; the buffer and the right-hand side are padded with zero rows
// to chord_rows(n) = round8(n) + 16, so the sweeps run over whole blocks of 8 rows and
// every prefetch stays inside the buffer without guards.
typedef __attribute__((address_space(3))) float lds_float;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x4 lds_f32x4;

__host__ __device__ constexpr int chord_rows(int n) { return ((n + 7) & ~7) + 16; }

// FP64 factor (padded column storage) -> FP32 rows, lanes of one wave over rows < n; the
// padding rows are zeroed once by the caller and never written here.
template <int BW>
__device__ void chord_to_f32(const double *Fp, int n, float *C_, int lane) {
  static_assert(BW <= 7, "FP32 chord rows hold 8 entries");
  constexpr int bp = BW + 1;
  const lds_double *F = (const lds_double *)Fp + BW * bp;
  lds_f32x4 *C = (lds_f32x4 *)C_;
  for (int j = lane; j < n; j += 64) {
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = t <= BW ? (float)F[j * bp + t] : 0.0f;
    C[2 * j] = f32x4{v[0], v[1], v[2], v[3]};
    C[2 * j + 1] = f32x4{v[4], v[5], v[6], v[7]};
  }
}

// Solve (L D L^T) x = x in FP32 by one lane.  Forward sweep right-looking: row j retires
// y_j from its accumulator and subtracts L(j + t, j) y_j from the next BW accumulators,
// so each row adds one dependent FMA to the critical path.  Backward sweep left-looking
// over the same rows: x_i = y_i / d_i - sum_t L(i + t, i) x_{i + t}, the x_{i + 1} term
// last.  Rows of the factor are loaded 8 rows ahead, x in blocks of 8 (two b128).
template <int BW>
__device__ __attribute__((noinline)) void chord_solve_f32(const float *C_, int n_, float *x_) {
  static_assert(BW <= 6, "the forward ring has 8 slots");
  const int n = __builtin_amdgcn_readfirstlane(n_);
  const int nb = (n + 7) & ~7;
  const lds_f32x4 *C = (const lds_f32x4 *)C_;
  lds_f32x4 *X = (lds_f32x4 *)x_;
  float acc[8], cf[8][8], xn[8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const f32x4 a = X[h], b = X[2 + h];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[4 * h + e] = a[e];
      xn[4 * h + e] = b[e];
    }
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const f32x4 a = C[2 * u], b = C[2 * u + 1];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      cf[u][e] = a[e];
      cf[u][4 + e] = b[e];
    }
  }
  for (int j0 = 0; j0 < nb; j0 += 8) {
    float ys[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float y = acc[u];
      ys[u] = y;
#pragma unroll
      for (int t = 1; t <= BW; ++t) acc[(u + t) & 7] = fmaf(-cf[u][t], y, acc[(u + t) & 7]);
      acc[u] = xn[u];
      const f32x4 a = C[2 * (j0 + u + 8)], b = C[2 * (j0 + u + 8) + 1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cf[u][e] = a[e];
        cf[u][4 + e] = b[e];
      }
    }
    X[j0 / 4] = f32x4{ys[0], ys[1], ys[2], ys[3]};
    X[j0 / 4 + 1] = f32x4{ys[4], ys[5], ys[6], ys[7]};
    const f32x4 a = X[j0 / 4 + 4], b = X[j0 / 4 + 5];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xn[e] = a[e];
      xn[4 + e] = b[e];
    }
  }
  // backward: block i0 = nb - 8, nb - 16, ..., rows i0 + 7 down to i0; xr[i & 7] holds x_i
  float xr[8], yv[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) xr[e] = 0.0f;
  {
    const f32x4 a = X[(nb - 8) / 4], b = X[(nb - 8) / 4 + 1];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      yv[e] = a[e];
      yv[4 + e] = b[e];
    }
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = nb - 1 - u;
    const f32x4 a = C[2 * i], b = C[2 * i + 1];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      cf[u][e] = a[e];
      cf[u][4 + e] = b[e];
    }
  }
  for (int i0 = nb - 8; i0 >= 0; i0 -= 8) {
    float yn[8];
    const int ip = i0 >= 8 ? i0 - 8 : 0;
    {
      const f32x4 a = X[ip / 4], b = X[ip / 4 + 1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        yn[e] = a[e];
        yn[4 + e] = b[e];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int s = 7 - u;  // i = i0 + s, i & 7 = s
      float acc2 = cf[u][0] * yv[s];
#pragma unroll
      for (int t = BW; t >= 2; --t) acc2 = fmaf(-cf[u][t], xr[(s + t) & 7], acc2);
      const float xi = fmaf(-cf[u][1], xr[(s + 1) & 7], acc2);
      xr[s] = xi;
      const int ic = i0 + s - 8 >= 0 ? i0 + s - 8 : 0;
      const f32x4 a = C[2 * ic], b = C[2 * ic + 1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cf[u][e] = a[e];
        cf[u][4 + e] = b[e];
      }
    }
    X[i0 / 4] = f32x4{xr[0], xr[1], xr[2], xr[3]};
    X[i0 / 4 + 1] = f32x4{xr[4], xr[5], xr[6], xr[7]};
#pragma unroll
    for (int e = 0; e < 8; ++e) yv[e] = yn[e];
  }
}

// Both take LDS pointers (passed as generic pointers): the cast makes every access inside an
// LDS instruction, whether or not the call is inlined.
template <int BW>
__device__ bool ldlt_serial(double *Fp, int n) {
  lds_double *F = (lds_double *)Fp;
  if constexpr (BW <= 6)
    return ldlt_serial_ring<BW>(F, n);
  else
    return ldlt_serial_shift<BW>(F, n);
}

template <int BW>
__device__ void ldlt_solve_serial(const double *Fp, int n, double *x) {
  const lds_double *F = (const lds_double *)Fp;
  lds_double *xl = (lds_double *)x;
  if constexpr (BW <= 6)
    ldlt_solve_ring<BW>(F, n, xl);
  else
    ldlt_solve_shift<BW>(F, n, xl);
}

}  // namespace
