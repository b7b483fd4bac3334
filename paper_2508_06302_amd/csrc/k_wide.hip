// Wide-band trajectory path of FSE-Shooting on gfx950 (Sec. 3.3 steps 2-3, App. E) for systems
// whose half bandwidth is beyond the fused kernel's and whose mass matrix is lumped (diagonal),
// such as the shell model of Sec. 4.3 (1872 DOF, half band 89).
//
// States (Eqs. E4-E7).  All trajectories of a call advance together, one kernel per phase of
// a step, the trajectory index in the lanes (layout [n][Wmax], trajectories contiguous).  The
// step equation (Eq. E6) S q + f_nl(q) = b_k is solved by a chord iteration on the linear step
// matrix S = w1^2 c0 M + w1 c2 D + K, which every trajectory of a continuation point shares:
// S^-1 is formed once per point in FP64, so each correction dq = S^-1 r is one dense FP64
// matrix-core GEMM over all trajectories of the point, while the residual r stays FP64 with the
// sparse polynomial forces.  The iteration contracts with ||S^-1 K_t||, the ratio of the
// nonlinear tangent to the step matrix (about 3e-6 on the shell at its linear response).
//
// Sensitivities (Eqs. E8-E9).  With T_{k+1} = S + K_t(q_{k+1}) the recursion
//   T Q' = w1^2 M (c0 Q + c1 U + A) + w1 D (c2 Q + U),  U' = c2 (Q' - Q) - U,
//   A' = c0 (Q' - Q) - c1 U - A
// is carried in the two combinations its right-hand side uses, P1 = c2 Q + U and
// P2 = c0 Q + c1 U + A (average acceleration: c3 = d1 = 1, d2 = 0, c1 c2 = 2 c0):
//   T Q' = w1^2 M P2 + w1 D P1,  P1' = 2 c2 Q' - P1,  P2' = (2 c0 + c1 c2) Q' - c1 P1 - P2,
// which is the same recursion (substitute U' and A'); at the last step Q = Q' and U = c2 Q' - P1.
// Two n x 2n arrays are read and written per step instead of three.  Per step and trajectory,
// T is assembled (batched over trajectories), factored as a banded LDL^T whose unit lower factor
// is written as 16 x 16 blocks (off-diagonal blocks negated, inverses of the diagonal blocks),
// and the right-hand side is swept forward and backward in 16-row blocks on the matrix cores
// (v_mfma_f64_16x16x4f64; v_mfma_f32_16x16x4f32 with FP32 storage in the mixed mode).
//
// Operand layout of both 16x16x4 instructions: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  The FP64 instruction holds D[4v + l / 16][l % 16] in element v, so a
// 16 x 16 tile held that way ("D layout") is also the B operand of four K-slices (slice v =
// element v).  The FP32 instruction holds D[4 (l / 16) + v][l % 16] instead; there, element v
// used as K-slice v supplies row sigma(4v + l/16) with sigma(4a + b) = 4b + a, so the A operands
// are read with their K index permuted by sigma (a product A D = (A sigma)(sigma D)) and tiles
// are loaded and stored with rows 4 (l / 16) + v.  Blocks of the factor and of D are stored in
// operand order: lane l of K-slice v reads entry v * 64 + l, which holds element
// (l % 16, 4v + l / 16) in FP64 and (l % 16, 4 (l / 16) + v) in FP32; LDS reads of operands are
// thereby contiguous across the wave (no bank conflicts).  The backward sweep needs the
// transposes of the blocks below the diagonal; they are transposed while staged into LDS.
#include <climits>
#include <cmath>
#include <cstring>

#include "fse_internal.h"

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct WideState {
  int n = 0, bw = 0, NB = 0, nrb = 0, nnz = 0;
  int span_r = 0, span_t = 0;   // LDS staging spans (rows) of the residual and tangent kernels
  int budget = 4;               // chord iterations launched per step (adapted from the last call)
  // device constants
  int32_t *rp = nullptr, *ci = nullptr;          // CSR pattern of M + D + K
  double *Mv = nullptr, *Dv = nullptr, *Kv = nullptr;
  double *mdiag = nullptr;                       // [n]
  double *Dfrag = nullptr;                       // [nrb][2NB+1][256]
  float *Dfrag32 = nullptr;
  uint32_t *Dmask = nullptr;                     // [nrb] nonzero D blocks
  int32_t *rlo = nullptr, *tlo = nullptr;        // first staged row per row / column block
  double *Kband = nullptr;                       // [n][bw+1] lower band of K (column-major)
  // per point
  double *Sv = nullptr;                          // [Bmax][nnz]
  double *Sband = nullptr;                       // [Bmax][n][bw+1]
  double *Sfac = nullptr;                        // [n][bw+1] factor scratch
  double *Sinv = nullptr;                        // [Bmax][n][n]
  // state chain, [n][Wmax] each
  double *u = nullptr, *a = nullptr, *bk = nullptr, *qh = nullptr, *r = nullptr;
  unsigned long long *acc = nullptr;             // [2][2][Wmax] max |dq|, max |q| (bits)
  int32_t *conv = nullptr;                       // [Wmax]
  double *ndprev = nullptr;                      // [Wmax]
  int32_t *ctl = nullptr;                        // [0] block ticket, [1] all converged, [2] budget hit
  // sensitivities: the tangent band, factor blocks and pivots of two steps in flight (the side
  // stream assembles and factors step k + 1 while the context stream sweeps step k)
  double *Tband = nullptr;                       // [2][Wmax][n][bw+1]
  void *frag = nullptr;                          // [2][Wmax][nrb][NB+1][256]
  void *dinv = nullptr;                          // [2][Wmax][nrb * 16]
  hipStream_t side = nullptr;
  hipEvent_t ev_fac[2] = {nullptr, nullptr}, ev_sw[2] = {nullptr, nullptr}, ev_go = nullptr;
  std::vector<hipEvent_t> ev_k;                  // start / end of every sweep of the last call
  int ev_used = 0;
  void *Ysc = nullptr;                           // [Wmax][n][2n]
  float *P32 = nullptr;                          // [Wmax][2n][2n] (mixed mode)
  size_t frag_bytes = 0, ysc_bytes = 0;
};

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kLanes = 64;        // trajectories per group of the batched state kernels
constexpr int kMaxNB = 6;         // 16-row blocks below the diagonal: half bandwidth <= 96
constexpr int kStageLds = 150 * 1024;

__device__ inline f64x4 mma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename FT> struct Vec4;
template <> struct Vec4<double> { typedef f64x4 T; };
template <> struct Vec4<float> { typedef f32x4 T; };

// Row of a 16 x 16 tile held by lane group g = l / 16 in element v (see the file header).
template <typename FT> __device__ inline int trow(int v, int g) { return sizeof(FT) == 8 ? 4 * v + g : 4 * g + v; }
// Operand-order position of element (row, col) of a 16 x 16 block, and its inverse.
template <typename FT> __host__ __device__ inline int opos(int row, int col) {
  return sizeof(FT) == 8 ? (col >> 2) * 64 + (col & 3) * 16 + row : (col & 3) * 64 + (col >> 2) * 16 + row;
}
template <typename FT> __device__ inline void opos_inv(int e, int &row, int &col) {
  const int v = e >> 6, l = e & 63;
  row = l & 15;
  col = sizeof(FT) == 8 ? 4 * v + (l >> 4) : 4 * (l >> 4) + v;
}

// forcing cosines (Eq. E1): forcing 0 has argument phi0 + phi1, forcing f >= 1 phi_{f+1,s} + rho phi1
__device__ inline double wforce(const double *F, int n, int e, int i, double phi1, const double *om,
                                const int32_t *sidx, const int32_t *Sdim, int St, int s, double phi0) {
  double v = F[i] * cos(phi0 + phi1);
  for (int f = 1; f < e; ++f) {
    const double ph = kTwoPi * (double)sidx[(f - 1) * St + s] / (double)Sdim[f - 1];
    v += F[(size_t)f * n + i] * cos(ph + om[f] / om[0] * phi1);
  }
  return v;
}

__device__ inline unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ inline double bitsd(unsigned long long v) { return __longlong_as_double((long long)v); }

// ------------------------------------------------------------------------------ per-point set-up
// Lower band of S = w1^2 c0 M + w1 c2 D + K (column-major [n][bw+1], entry (m + r, m) at m (bw+1) + r)
// and S on the CSR pattern.  Full-row bands [n][2bw+1] hold entry (i, j) at i (2bw+1) + j - i + bw.
__global__ void k_wide_sband(const double *__restrict__ Mb, const double *__restrict__ Db,
                             const double *__restrict__ Kb, const double *__restrict__ omega, int d, int n,
                             int bw, double c0, double c2, double *__restrict__ Sband,
                             const double *__restrict__ Mv, const double *__restrict__ Dv,
                             const double *__restrict__ Kv, int nnz, double *__restrict__ Sv) {
  const int b = blockIdx.y;
  const double w1 = omega[b * d];
  const int P = bw + 1, W2 = 2 * bw + 1;
  const size_t nb = (size_t)n * P;
  for (size_t pos = (size_t)blockIdx.x * blockDim.x + threadIdx.x; pos < nb; pos += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(pos / P), r = (int)(pos - (size_t)m * P), i = m + r;
    double v = 0.0;
    if (i < n) {
      const size_t e = (size_t)i * W2 + (bw - r);
      v = w1 * w1 * c0 * Mb[e] + w1 * c2 * Db[e] + Kb[e];
    }
    Sband[b * nb + pos] = v;
  }
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += gridDim.x * blockDim.x)
    Sv[(size_t)b * nnz + p] = w1 * w1 * c0 * Mv[p] + w1 * c2 * Dv[p] + Kv[p];
}

// ------------------------------------------------------------------------------ banded LDL^T
// Right-looking LDL^T of one symmetric band (column-major lower band In [n][bw+1]) per block,
// the bw + 1 active columns held in an LDS ring (slot j mod (bw+1)); 256 threads share the
// bw (bw + 1) / 2 updates of each column, two barriers per column.
// OUT == 0: the scaled factor (d_j, l_{j+r,j}) written back as a band to Out [n][bw+1].
// OUT == 1: 16 x 16 blocks of the unit lower factor for the sweeps: for row block I, slots
//           s = 0..NB-1 hold -L(I, I - NB + s) and slot NB holds L(I, I)^-1, all in forward-
//           fragment order, FT precision; dinv [nrb * 16] holds 1 / d (1 on padded rows).
constexpr int kFacThreads = 256;
constexpr int kMaxPairs = 19;  // ceil(96 * 97 / 2 / 256)

template <int OUT, typename FT>
__global__ __launch_bounds__(kFacThreads) void k_wide_factor(const double *__restrict__ In, size_t in_stride,
                                                             int n, int bw, int NB, int nrb,
                                                             double *__restrict__ Out, FT *__restrict__ frag,
                                                             FT *__restrict__ dinv, DevStatus *st) {
  extern __shared__ double lds[];
  const int P = bw + 1;
  double *ring = lds;                      // [P][P]
  double *blk = ring + (size_t)P * P;      // [NB+1][16][16] row-major, block column being built
  double *inv = blk + (size_t)(NB + 1) * 256;  // [16][16] inverse of the diagonal block
  const int tid = threadIdx.x;
  const size_t w = blockIdx.x;
  const double *T = In + w * in_stride;
  const size_t fstride = (size_t)nrb * (NB + 1) * 256;
  FT *fw = frag + w * fstride;
  FT *dw = dinv + w * (size_t)nrb * 16;
  // this thread's (r, c) pairs, 1 <= c <= r <= bw, packed r | c << 8
  int pr[kMaxPairs];
  int np = 0;
  {
    const int npairs = bw * (bw + 1) / 2;
    int p = tid, r = 1, c = 1;
    // walk the pairs in order (r, c) = (1,1), (2,1), (2,2), (3,1) ... and keep every 256th
    for (int q = 0; q < npairs && np < kMaxPairs; ++q) {
      if (q == p) {
        pr[np++] = r | (c << 8);
        p += kFacThreads;
      }
      if (++c > r) {
        ++r;
        c = 1;
      }
    }
  }
  for (int e = tid; e < P * P; e += kFacThreads) {
    const int c = e / P;
    ring[e] = c < n ? T[(size_t)c * P + (e - c * P)] : 0.0;
  }
  if (OUT == 1) {
    for (int e = tid; e < (NB + 1) * 256; e += kFacThreads) blk[e] = (e < 256 && (e >> 4) == (e & 15)) ? 1.0 : 0.0;
  }
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    const int s = j % P;
    const double dj = ring[s * P];
    if (!(dj != 0.0) || !isfinite(dj)) bad = true;
    const double id = 1.0 / dj;
#pragma unroll
    for (int k = 0; k < kMaxPairs; ++k) {
      if (k < np) {
        const int r = pr[k] & 255, c = pr[k] >> 8;
        if (j + r < n) {
          int sc = s + c;
          if (sc >= P) sc -= P;
          ring[sc * P + (r - c)] -= ring[s * P + r] * ring[s * P + c] * id;
        }
      }
    }
    __syncthreads();
    if (tid <= bw) {
      const int r = tid;
      const double v = ring[s * P + r];
      if (OUT == 0) {
        Out[(size_t)j * P + r] = r == 0 ? v : v * id;
      } else if (r == 0) {
        dw[j] = (FT)id;
      } else if (j + r < n) {
        const int i = j + r, I = i >> 4, J = j >> 4;
        blk[(I - J) * 256 + (i & 15) * 16 + (j & 15)] = v * id;
      }
      const int nx = j + P;
      ring[s * P + r] = nx < n ? T[(size_t)nx * P + r] : 0.0;
    }
    __syncthreads();
    if (OUT == 1 && ((j & 15) == 15 || j == n - 1)) {
      const int J = j >> 4;
      // inverse of the unit lower diagonal block, one column per thread
      if (tid < 16) {
        const int c = tid;
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          double v = r == c ? 1.0 : 0.0;
#pragma unroll
          for (int k = 0; k < r; ++k)
            if (k >= c) v -= blk[r * 16 + k] * x[k];
          x[r] = r < c ? 0.0 : v;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) inv[r * 16 + c] = x[r];
      }
      __syncthreads();
      {
        // operand-order position e holds element (row, cc)
        const int e = tid;
        int row, cc;
        opos_inv<FT>(e, row, cc);
        fw[((size_t)J * (NB + 1) + NB) * 256 + e] = (FT)inv[row * 16 + cc];
        for (int t = 1; t <= NB; ++t) {
          const int I = J + t;
          if (I >= nrb) break;
          fw[((size_t)I * (NB + 1) + (NB - t)) * 256 + e] = (FT)(-blk[t * 256 + row * 16 + cc]);
        }
      }
      __syncthreads();
      for (int e = tid; e < (NB + 1) * 256; e += kFacThreads) blk[e] = (e < 256 && (e >> 4) == (e & 15)) ? 1.0 : 0.0;
      __syncthreads();
    }
  }
  if (OUT == 1)
    for (int i = n + tid; i < nrb * 16; i += kFacThreads) dw[i] = (FT)1.0;
  if (bad && tid == 0) atomicOr(&st->flags, (int)DEV_SINGULAR);
}

// S^-1 = (L D L^T)^-1 column by column from the band factor F [n][bw+1] (OUT == 0 above):
// thread c solves for e_c, using its column of the row-major output as the work vector.
__global__ void k_wide_sinv(const double *__restrict__ F, int n, int bw, double *__restrict__ X) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int P = bw + 1;
  for (int i = 0; i < n; ++i) {
    double y = i == c ? 1.0 : 0.0;
    if (i > c) {
      const int t0 = i < bw ? i : bw;
      for (int t = 1; t <= t0; ++t) y -= F[(size_t)(i - t) * P + t] * X[(size_t)(i - t) * n + c];
    }
    X[(size_t)i * n + c] = y;
  }
  for (int i = n - 1; i >= 0; --i) {
    double x = X[(size_t)i * n + c] / F[(size_t)i * P];
    const int t1 = (n - 1 - i) < bw ? (n - 1 - i) : bw;
    for (int t = 1; t <= t1; ++t) x -= F[(size_t)i * P + t] * X[(size_t)(i + t) * n + c];
    X[(size_t)i * n + c] = x;
  }
}

// ------------------------------------------------------------------------------ state chain
struct WideSys {
  const int32_t *rp, *ci;
  const double *Dv, *Kv, *Sv, *mdiag, *F;
  const int32_t *f2_ptr, *f2_jk;
  const double *f2_v;
  const int32_t *f3_ptr, *f3_jkl;
  const double *f3_v;
  int n, nnz, e, d, St, W, ldw;
};

// reset of the status word and the chord control of a state pass
__global__ void k_reset_status_wide(DevStatus *st, int32_t *ctl) {
  if (threadIdx.x == 0) {
    st->flags = 0;
    st->first_step = INT_MAX;
    st->max_iters = 0;
    st->pad = 0;
    st->total_iters = 0ull;
    ctl[0] = 0;
    ctl[1] = 0;
    ctl[2] = 0;
  }
}

// consistent a_0 (Eq. E2 at phi_1 = 0): w1^2 m_i a_i = e_0 - w1 (D u_0)_i - (K q_0)_i - f_nl(q_0)_i
__global__ void k_wide_init(WideSys sy, const double *__restrict__ omega, const int32_t *__restrict__ sidx,
                            const int32_t *__restrict__ Sdim, double phib, const double *__restrict__ q0,
                            const double *__restrict__ u0, double *__restrict__ u, double *__restrict__ a) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
  if (w >= sy.W) return;
  const int ld = sy.ldw, b = w / sy.St, s = w - b * sy.St;
  const double *om = omega + b * sy.d;
  const double w1 = om[0];
  double v = wforce(sy.F, sy.n, sy.e, i, 0.0, om, sidx, Sdim, sy.St, s, phib * b);
  for (int p = sy.rp[i]; p < sy.rp[i + 1]; ++p) {
    const int j = sy.ci[p];
    v -= w1 * sy.Dv[p] * u0[(size_t)j * ld + w] + sy.Kv[p] * q0[(size_t)j * ld + w];
  }
  for (int p = sy.f2_ptr[i]; p < sy.f2_ptr[i + 1]; ++p)
    v -= sy.f2_v[p] * q0[(size_t)sy.f2_jk[2 * p] * ld + w] * q0[(size_t)sy.f2_jk[2 * p + 1] * ld + w];
  for (int p = sy.f3_ptr[i]; p < sy.f3_ptr[i + 1]; ++p)
    v -= sy.f3_v[p] * q0[(size_t)sy.f3_jkl[3 * p] * ld + w] * q0[(size_t)sy.f3_jkl[3 * p + 1] * ld + w] *
         q0[(size_t)sy.f3_jkl[3 * p + 2] * ld + w];
  a[(size_t)i * ld + w] = v / (w1 * w1 * sy.mdiag[i]);
  u[(size_t)i * ld + w] = u0[(size_t)i * ld + w];
}

// b_k (Eq. E7) and the predictor q_k + h u_k + h^2/2 a_k; resets the chord state of the step
__global__ void k_wide_predict(WideSys sy, TrajParams P, int k, const double *__restrict__ omega,
                               const int32_t *__restrict__ sidx, const int32_t *__restrict__ Sdim,
                               const double *__restrict__ q, const double *__restrict__ u,
                               const double *__restrict__ a, double *__restrict__ bk, double *__restrict__ qh,
                               unsigned long long *__restrict__ acc, int32_t *__restrict__ conv,
                               double *__restrict__ ndprev, int32_t *__restrict__ ctl) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
  if (w >= sy.W) return;
  const int ld = sy.ldw, b = w / sy.St, s = w - b * sy.St;
  const double *om = omega + b * sy.d;
  const double w1 = om[0];
  const size_t o = (size_t)i * ld + w;
  double v = wforce(sy.F, sy.n, sy.e, i, (double)(k + 1) * P.h, om, sidx, Sdim, sy.St, s, P.phib * b);
  v += w1 * w1 * sy.mdiag[i] * (P.c0 * q[o] + P.c1 * u[o] + a[o]);
  double dd = 0.0;
  for (int p = sy.rp[i]; p < sy.rp[i + 1]; ++p) {
    const size_t oj = (size_t)sy.ci[p] * ld + w;
    dd += sy.Dv[p] * (P.c2 * q[oj] + u[oj]);
  }
  bk[o] = v + w1 * dd;
  qh[o] = q[o] + P.h * u[o] + 0.5 * P.h * P.h * a[o];
  if (i == 0) {
    acc[w] = 0ull;
    acc[ld + w] = 0ull;
    conv[w] = 0;
    ndprev[w] = INFINITY;
    if (w == 0) {
      ctl[0] = 0;
      ctl[1] = 0;
    }
  }
}

// r = S qh + f_nl(qh) - b for a block of rows and a group of 64 trajectories, the rows of qh the
// block reads staged in LDS (span rows from rlo[block]).  One wave per row: the staged rows
// (about 100 KB for the shell's band) allow one block per CU, so the block carries 16 waves.
// The term lists of a row are wave-uniform (scalar loads); they are walked eight terms at a
// time, all index and value loads and LDS reads of the eight issued before their products, so
// that their latencies overlap instead of adding up term by term.  The sum runs in list order.
constexpr int kResRows = 16;
constexpr int kResThreads = 64 * kResRows;
constexpr int kTermBatch = 8;

// The term lists never change while a kernel runs; read through the constant address space, a
// wave-uniform address compiles to scalar loads (the barrier before the row loop would otherwise
// keep the compiler from proving them unclobbered, and it would use vector loads).
template <class T>
using const_as = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ const_as<T> as_const(const T *p) {
  return (const_as<T>)p;
}

__device__ __forceinline__ double res_lin(const_as<double> val, const_as<int32_t> ci, int p, int e,
                                          const double *__restrict__ sq, int lo, int lane, double v) {
  for (; p + kTermBatch <= e; p += kTermBatch) {
    double a[kTermBatch], x[kTermBatch];
    int c[kTermBatch];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) c[t] = ci[p + t];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) a[t] = val[p + t];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) x[t] = sq[(c[t] - lo) * kLanes + lane];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) v += a[t] * x[t];
  }
  for (; p < e; ++p) v += val[p] * sq[(ci[p] - lo) * kLanes + lane];
  return v;
}

__device__ __forceinline__ double res_quad(const_as<double> val, const_as<int32_t> jk, int p, int e,
                                           const double *__restrict__ sq, int lo, int lane, double v) {
  for (; p + kTermBatch <= e; p += kTermBatch) {
    double a[kTermBatch], x[kTermBatch], y[kTermBatch];
    int c[2 * kTermBatch];
#pragma unroll
    for (int t = 0; t < 2 * kTermBatch; ++t) c[t] = jk[2 * p + t];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) a[t] = val[p + t];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) {
      x[t] = sq[(c[2 * t] - lo) * kLanes + lane];
      y[t] = sq[(c[2 * t + 1] - lo) * kLanes + lane];
    }
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) v += a[t] * x[t] * y[t];
  }
  for (; p < e; ++p) v += val[p] * sq[(jk[2 * p] - lo) * kLanes + lane] * sq[(jk[2 * p + 1] - lo) * kLanes + lane];
  return v;
}

__device__ __forceinline__ double res_cub(const_as<double> val, const_as<int32_t> jkl, int p, int e,
                                          const double *__restrict__ sq, int lo, int lane, double v) {
  for (; p + kTermBatch <= e; p += kTermBatch) {
    double a[kTermBatch], x[kTermBatch], y[kTermBatch], z[kTermBatch];
    int c[3 * kTermBatch];
#pragma unroll
    for (int t = 0; t < 3 * kTermBatch; ++t) c[t] = jkl[3 * p + t];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) a[t] = val[p + t];
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) {
      x[t] = sq[(c[3 * t] - lo) * kLanes + lane];
      y[t] = sq[(c[3 * t + 1] - lo) * kLanes + lane];
      z[t] = sq[(c[3 * t + 2] - lo) * kLanes + lane];
    }
#pragma unroll
    for (int t = 0; t < kTermBatch; ++t) v += a[t] * x[t] * y[t] * z[t];
  }
  for (; p < e; ++p)
    v += val[p] * sq[(jkl[3 * p] - lo) * kLanes + lane] * sq[(jkl[3 * p + 1] - lo) * kLanes + lane] *
         sq[(jkl[3 * p + 2] - lo) * kLanes + lane];
  return v;
}

__global__ __launch_bounds__(kResThreads) void k_wide_resid(WideSys sy, const int32_t *__restrict__ rlo, int span,
                                                            const double *__restrict__ qh,
                                                            const double *__restrict__ bk, double *__restrict__ r,
                                                            const int32_t *__restrict__ conv,
                                                            const int32_t *__restrict__ ctl) {
  extern __shared__ double sq[];
  if (ctl[1]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w0 = blockIdx.y * kLanes, w = w0 + lane;
  const bool act = w < sy.W && !conv[w];
  if (!__syncthreads_or(act)) return;
  const int ld = sy.ldw, i0 = blockIdx.x * kResRows, lo = rlo[blockIdx.x];
  for (int e = threadIdx.x; e < span * kLanes; e += blockDim.x) {
    const int j = lo + e / kLanes, ww = w0 + (e & 63);
    sq[e] = (j < sy.n && ww < sy.W) ? qh[(size_t)j * ld + ww] : 0.0;
  }
  __syncthreads();
  const int i = __builtin_amdgcn_readfirstlane(i0 + wv);  // wave-uniform: index lists load as scalars
  if (i >= sy.n) return;
  // the point of this group's trajectories: uniform over the wave whenever S~ is a multiple of 64
  const int b = __builtin_amdgcn_readfirstlane((w0 < sy.W ? w0 : sy.W - 1) / sy.St);
  const int bl = (w < sy.W ? w : sy.W - 1) / sy.St;
  const_as<int32_t> rp = as_const(sy.rp), p2 = as_const(sy.f2_ptr), p3 = as_const(sy.f3_ptr);
  double v;
  if (__builtin_amdgcn_ballot_w64(bl != b) == 0) {
    v = res_lin(as_const(sy.Sv + (size_t)b * sy.nnz), as_const(sy.ci), rp[i], rp[i + 1], sq, lo, lane, 0.0);
  } else {
    // trajectories of two points in one group: the step-matrix values per lane
    const double *Sv = sy.Sv + (size_t)bl * sy.nnz;
    v = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) v += Sv[p] * sq[(sy.ci[p] - lo) * kLanes + lane];
  }
  v = res_quad(as_const(sy.f2_v), as_const(sy.f2_jk), p2[i], p2[i + 1], sq, lo, lane, v);
  v = res_cub(as_const(sy.f3_v), as_const(sy.f3_jkl), p3[i], p3[i + 1], sq, lo, lane, v);
  if (w < sy.W) r[(size_t)i * ld + w] = v - bk[(size_t)i * ld + w];
}

// dq = S^-1 r per point (FP64 matrix cores: one wave per 16 rows x 16 trajectories, K = n),
// qh -= dq for the trajectories still iterating, and the per-trajectory maxima of |dq| and |qh|.
// The last block to finish decides convergence for every trajectory and prepares the next
// iteration's accumulators.  Stop rule (the per-step stop of the oracle, tightened): the last
// update below 1e-2 tol ||q||_inf, or the FP64 noise floor (an update below tol ||q||_inf that no
// longer halves).  No geometric extrapolation from the ratio of successive updates: with a lumped
// mass whose entries span orders of magnitude, S^-1 K_t is far from normal and that ratio
// underestimates the next update.
constexpr int kChordKSplit = 4;                    // waves per 16 x 16 tile, one K range each
constexpr int kChordThreads = 256 * kChordKSplit;  // 4 row blocks x kChordKSplit waves
constexpr int kChordBatch = 8;                     // K steps whose loads are issued together

__global__ __launch_bounds__(kChordThreads) void k_wide_chord(int n, int W, int St, int ldw, int ntile_pt,
                                                    const double *__restrict__ Sinv, const double *__restrict__ r,
                                                    double *__restrict__ qh, unsigned long long *__restrict__ acc,
                                                    int32_t *__restrict__ conv, double *__restrict__ ndprev,
                                                    int32_t *__restrict__ ctl, int it, int last_it, int final_budget,
                                                    int k, double tol, DevStatus *st) {
  if (ctl[1]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rsub = wv & 3, kc = wv >> 2;                 // row block within the block, K range
  const int b = blockIdx.y / ntile_pt, ct = blockIdx.y - b * ntile_pt;
  const int col = ct * 16 + (lane & 15);                 // trajectory within the point
  const int w = b * St + col;
  const bool valid = col < St && w < W;
  const bool act = valid && !conv[w];
  unsigned long long *accA = acc + (size_t)(it & 1) * 2 * ldw;
  const int rb = blockIdx.x * 4 + rsub;                  // 16-row block of this wave
  __shared__ f64x4 part[kChordKSplit - 1][4][64];        // partial tiles of K ranges 1..
  const bool any = __syncthreads_or(act);
  f64x4 c = {0.0, 0.0, 0.0, 0.0};
  if (any) {
    const double *A = Sinv + (size_t)b * n * n;
    const int arow = rb * 16 + (lane & 15);
    const bool arow_ok = arow < n;
    // clamped indices: every load is in bounds and unconditional, operands outside are zeroed
    const int arc = min(arow, n - 1), wc = min(w, W - 1);
    const int nk = (n + 3) / 4, per = (nk + kChordKSplit - 1) / kChordKSplit;
    const int s1 = min(nk, (kc + 1) * per);
    int ks = kc * per;
    // S^-1 is symmetric: A[arow][kk] is read as A[kk][arow] (16 consecutive rows per k)
    for (; ks + kChordBatch <= s1; ks += kChordBatch) {
      double av[kChordBatch], bv[kChordBatch];
#pragma unroll
      for (int t = 0; t < kChordBatch; ++t) {
        const int kk = 4 * (ks + t) + (lane >> 4), kq = min(kk, n - 1);
        av[t] = A[(size_t)kq * n + arc];
        bv[t] = r[(size_t)kq * ldw + wc];
        if (!(arow_ok && kk < n)) av[t] = 0.0;
        if (!(valid && kk < n)) bv[t] = 0.0;
      }
#pragma unroll
      for (int t = 0; t < kChordBatch; ++t) c = mma(av[t], bv[t], c);
    }
    for (; ks < s1; ++ks) {
      const int kk = 4 * ks + (lane >> 4), kq = min(kk, n - 1);
      double av = A[(size_t)kq * n + arc], bv = r[(size_t)kq * ldw + wc];
      if (!(arow_ok && kk < n)) av = 0.0;
      if (!(valid && kk < n)) bv = 0.0;
      c = mma(av, bv, c);
    }
    if (kc > 0) part[kc - 1][rsub][lane] = c;
  }
  __syncthreads();
  if (any && kc == 0) {
    // the K ranges in order
#pragma unroll
    for (int q = 0; q < kChordKSplit - 1; ++q) {
      const f64x4 pq = part[q][rsub][lane];
#pragma unroll
      for (int v = 0; v < 4; ++v) c[v] += pq[v];
    }
    double md = 0.0, mq = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rb * 16 + 4 * v + (lane >> 4);
      if (act && row < n) {
        const size_t o = (size_t)row * ldw + w;
        const double qn = qh[o] - c[v];
        qh[o] = qn;
        md = fmax(md, fabs(c[v]));
        mq = fmax(mq, fabs(qn));
        if (!(c[v] == c[v])) md = NAN;
      }
    }
    // lanes l, l + 16, l + 32, l + 48 hold the same trajectory
    for (int o = 16; o < 64; o <<= 1) {
      const double x = __shfl_xor(md, o), y = __shfl_xor(mq, o);
      md = (md != md || x != x) ? NAN : fmax(md, x);
      mq = fmax(mq, y);
    }
    if (act && lane < 16) {
      atomicMax(&accA[w], dbits(md != md ? INFINITY : md));
      atomicMax(&accA[ldw + w], dbits(mq));
    }
  }
  // last block: decisions for every trajectory of the call
  __threadfence();
  __shared__ int ticket;
  if (threadIdx.x == 0) ticket = atomicAdd(&ctl[0], 1);
  __syncthreads();
  if (ticket != (int)(gridDim.x * gridDim.y) - 1) return;
  __threadfence();
  unsigned long long *accN = acc + (size_t)((it + 1) & 1) * 2 * ldw;
  int unconv = 0, maxit = 0;
  unsigned long long tot = 0;
  for (int ww = threadIdx.x; ww < W; ww += blockDim.x) {
    accN[ww] = 0ull;
    accN[ldw + ww] = 0ull;
    if (conv[ww]) continue;
    const double nd = bitsd(atomicAdd(&accA[ww], 0ull)), nq = bitsd(atomicAdd(&accA[ldw + ww], 0ull));
    const double prev = ndprev[ww];
    bool done = false;
    if (!(nd < INFINITY)) {
      atomicOr(&st->flags, (int)DEV_NAN);
      done = true;
    } else if (nd <= 1e-2 * tol * nq || (nd <= tol * nq && nd > 0.5 * prev)) {
      done = true;
    }
    ndprev[ww] = nd;
    if (!done && it == last_it) {
      // the launched iterations ran out: a retry with the full budget, or NOCONV after it
      atomicOr(&ctl[2], 1);
      atomicMin(&st->first_step, k);
      if (final_budget) atomicOr(&st->flags, (int)DEV_NOCONV);
      done = true;
    }
    if (done) {
      conv[ww] = 1;
      maxit = max(maxit, it + 1);
      tot += (unsigned long long)(it + 1);
    } else {
      ++unconv;
    }
  }
  // block reduction of the counts
  __shared__ int s_un, s_mx;
  __shared__ unsigned long long s_tot;
  if (threadIdx.x == 0) {
    s_un = 0;
    s_mx = 0;
    s_tot = 0ull;
  }
  __syncthreads();
  atomicAdd(&s_un, unconv);
  atomicMax(&s_mx, maxit);
  atomicAdd(&s_tot, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_un == 0) ctl[1] = 1;
    if (s_mx > 0) atomicMax(&st->max_iters, s_mx);
    if (s_tot) atomicAdd(&st->total_iters, s_tot);
    ctl[0] = 0;
  }
}

// Eq. (E5): u_{k+1} = c2 (q_{k+1} - q_k) - u_k, a_{k+1} = c0 (q_{k+1} - q_k) - c1 u_k - a_k
__global__ void k_wide_update(int n, int W, int ldw, TrajParams P, const double *__restrict__ qh,
                              const double *__restrict__ q, double *__restrict__ qn, double *__restrict__ u,
                              double *__restrict__ a, int last, double *__restrict__ zT, DevStatus *st) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
  if (w >= W) return;
  const size_t o = (size_t)i * ldw + w;
  const double x = qh[o], dq = x - q[o], uo = u[o];
  const double un = P.c2 * dq - uo;
  a[o] = P.c0 * dq - P.c1 * uo - a[o];
  u[o] = un;
  qn[o] = x;
  if (last) {
    zT[o] = x;
    zT[(size_t)(n + i) * ldw + w] = un;
    if (!isfinite(x) || !isfinite(un)) atomicOr(&st->flags, (int)DEV_NAN);
  }
}

// ------------------------------------------------------------------------------ sensitivities
// Lower band of Base + K_t(q) for every trajectory (Base = S of its point, or K for A_0), out
// [W][n][bw+1].  Block: 16 band columns x 64 trajectories; the rows of q the tangent lists read
// are staged in LDS; 64 band positions at a time are formed (one position per wave iteration,
// trajectories in the lanes) and written out transposed, each trajectory's positions contiguous.
__global__ __launch_bounds__(256) void k_wide_tangent(int n, int bw, int W, int St, int ldw,
                                                      const int32_t *__restrict__ tlo, int span,
                                                      const double *__restrict__ q,
                                                      const int32_t *__restrict__ kt_ptr,
                                                      const int32_t *__restrict__ kt_idx,
                                                      const double *__restrict__ kt_c,
                                                      const double *__restrict__ base, size_t base_stride,
                                                      double *__restrict__ T) {
  extern __shared__ double lds[];
  double *sq = lds;                                  // [span][64]
  double *tile = lds + (size_t)span * kLanes;        // [64][65]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int P = bw + 1, m0 = blockIdx.x * 16, w0 = blockIdx.y * kLanes, lo = tlo[blockIdx.x];
  for (int e = threadIdx.x; e < span * kLanes; e += blockDim.x) {
    const int j = lo + e / kLanes, ww = w0 + (e & 63);
    sq[e] = (j < n && ww < W) ? q[(size_t)j * ldw + ww] : 0.0;
  }
  __syncthreads();
  const int p0 = m0 * P, p1 = min(m0 + 16, n) * P;
  const size_t nb = (size_t)n * P;
  for (int c0 = p0; c0 < p1; c0 += 64) {
    for (int pl = wv; pl < 64; pl += 4) {
      const int pos = __builtin_amdgcn_readfirstlane(c0 + pl);
      double v = 0.0;
      if (pos < p1)
        for (int p = kt_ptr[pos]; p < kt_ptr[pos + 1]; ++p) {
          const int ia = kt_idx[2 * p], ib = kt_idx[2 * p + 1];
          const double ya = sq[(ia - lo) * kLanes + lane];
          v += kt_c[p] * ya * (ib >= 0 ? sq[(ib - lo) * kLanes + lane] : 1.0);
        }
      tile[pl * 65 + lane] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
      const int wl = e >> 6, pl = e & 63, pos = c0 + pl, ww = w0 + wl;
      if (pos < p1 && ww < W)
        T[(size_t)ww * nb + pos] = base[(size_t)(ww / St) * base_stride + pos] + tile[pl * 65 + wl];
    }
    __syncthreads();
  }
}

// P1_0 = c2 Q_0 + U_0 = [c2 I, I], P2_0 = c0 Q_0 + c1 U_0 + A_0 = [c0 I, c1 I] + A_0 with
// A_0 = -(w1^2 M)^-1 [K + K_t(q_0), w1 D]: rows 0..n-1 of Pbuf[w] hold P1, rows n..2n-1 P2.
template <typename FT>
__global__ void k_wide_sens0(int n, int bw, int W, int St, int d, TrajParams P, const double *__restrict__ omega,
                             const double *__restrict__ KT, const double *__restrict__ Db,
                             const double *__restrict__ mdiag, FT *__restrict__ Pbuf) {
  const int n2 = 2 * n, Pb = bw + 1, W2 = 2 * bw + 1;
  const size_t w = blockIdx.y;
  const int row = blockIdx.x;  // 0 .. 2n-1
  if ((int)w >= W) return;
  const double w1 = omega[(w / St) * d];
  const double *kt = KT + w * (size_t)n * Pb;
  FT *out = Pbuf + (w * n2 + row) * n2;
  for (int j = threadIdx.x; j < n2; j += blockDim.x) {
    double v = 0.0;
    if (row < n) {
      const int i = row;
      v = (j == i ? P.c2 : 0.0) + (j == n + i ? 1.0 : 0.0);
    } else {
      const int i = row - n;
      v = (j == i ? P.c0 : 0.0) + (j == n + i ? P.c1 : 0.0);
      const double s = -1.0 / (w1 * w1 * mdiag[i]);
      if (j < n) {
        const int dij = i - j;
        if (dij >= 0 && dij <= bw) v += s * kt[(size_t)j * Pb + dij];
        else if (dij < 0 && -dij <= bw) v += s * kt[(size_t)i * Pb - dij];
      } else {
        const int jj = j - n;
        if (abs(jj - i) <= bw) v += s * w1 * Db[(size_t)i * W2 + (jj - i + bw)];
      }
    }
    out[j] = (FT)v;
  }
}

// One sensitivity step (see the file header) for a 64-column group of one trajectory: four waves,
// one 16-column tile each.  Forward: for row blocks I = 0..nrb-1,
//   acc = w1 sum_J D(I,J) P1_J + w1^2 m_I P2_I  -  sum_{J<I} L(I,J) Y_J,   Y_I = L(I,I)^-1 acc,
// storing Z_I = D_I^-1 Y_I; backward for I = nrb-1..0:
//   acc = Z_I - sum_{J>I} L(J,I)^T X_J,   X_I = L(I,I)^-T acc,
// then P1, P2 of block I are replaced (or Q, U at the last step).  The factor and D blocks of a
// row block are staged in LDS for the four waves; P1 blocks I-NB..I+NB and the last NB solution
// blocks stay in registers (D layout).  Blocks map to XCDs by trajectory, so the column groups of
// a trajectory share its factor in one L2.
template <int NB, typename FT, bool EXACT>
__global__ __launch_bounds__(256, 2) void k_wide_sweep(int n, int W, int St, int d, int nrb, int ncg, int per_xcd,
                                                    const double *__restrict__ omega, TrajParams P,
                                                    const double *__restrict__ mdiag,
                                                    const FT *__restrict__ Dfrag, const uint32_t *__restrict__ Dmask,
                                                    const FT *__restrict__ frag, const FT *__restrict__ dinv,
                                                    FT *__restrict__ Pbuf, FT *__restrict__ Ysc, int last) {
  typedef typename Vec4<FT>::T V4;
  constexpr int NBL = 2 * NB + 1;               // D blocks per row block
  constexpr int NSTG = NB + 1 + NBL;            // staged blocks per forward row block
  __shared__ FT stg[NSTG * 256];
  __shared__ FT stgr[32];                       // per-row scalars of the block: mass, 1 / d
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int pidx = xcd * per_xcd + slot;
  if (pidx >= W * ncg) return;
  const int w = pidx / ncg, cg = pidx - w * ncg;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n2 = 2 * n;
  const int c0 = (cg * 4 + wv) * 16;
  const int col = c0 + (lane & 15);
  const bool colok = col < n2;
  const int rsub = lane >> 4;                   // row within a 4-row slice
  const double w1 = omega[(w / St) * d];
  const FT fw1 = (FT)w1, fw1s = (FT)(w1 * w1);
  const size_t fst = (size_t)(NB + 1) * 256;
  const FT *fr = frag + (size_t)w * nrb * fst;
  const FT *dv = dinv + (size_t)w * nrb * 16;
  FT *P1 = Pbuf + (size_t)w * n2 * n2;
  FT *P2 = P1 + (size_t)n * n2;
  FT *Y = Ysc + (size_t)w * n * n2;
  const V4 zero4 = {0, 0, 0, 0};

  // EXACT: n and 2n are multiples of 16, so every row of a block exists and a 16-column tile is
  // either whole or absent (a wave-uniform test)
  const bool wave_cols = c0 < n2;
  const FT *colp = nullptr;
  auto ld4 = [&](const FT *base, int I) -> V4 {
    V4 r = zero4;
    if (EXACT) {
      if (I >= 0 && I < nrb && wave_cols) {
        const FT *b = base + (size_t)(I * 16) * n2 + col;
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = b[(size_t)trow<FT>(v, rsub) * n2];
      }
    } else if (I >= 0 && I < nrb && colok) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = I * 16 + trow<FT>(v, rsub);
        if (row < n) r[v] = base[(size_t)row * n2 + col];
      }
    }
    return r;
  };
  auto st4 = [&](FT *base, int I, V4 x) {
    if (EXACT) {
      if (!wave_cols) return;
      FT *b = base + (size_t)(I * 16) * n2 + col;
#pragma unroll
      for (int v = 0; v < 4; ++v) b[(size_t)trow<FT>(v, rsub) * n2] = x[v];
      return;
    }
    if (!colok) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = I * 16 + trow<FT>(v, rsub);
      if (row < n) base[(size_t)row * n2 + col] = x[v];
    }
  };
  (void)colp;

  // ---------------- forward sweep
  V4 p1w[NBL];
#pragma unroll
  for (int s = 0; s < NBL; ++s) p1w[s] = ld4(P1, s - NB);
  V4 yw[NB];
#pragma unroll
  for (int s = 0; s < NB; ++s) yw[s] = zero4;
  // staged blocks of row block I: [0, NB] factor slots, [NB + 1, NB + NBL] D blocks
  FT pre[NSTG];
#pragma unroll
  for (int s = 0; s <= NB; ++s) pre[s] = fr[s * 256 + tid];
#pragma unroll
  for (int s = 0; s < NBL; ++s) pre[NB + 1 + s] = Dfrag[s * 256 + tid];
  // per-row scalars of a block (lumped mass, 1/d of the factor), staged with the blocks by the
  // first 32 threads
  auto ldrow = [&](int I) -> FT {
    if (tid < 16) {
      const int row = I * 16 + tid;
      return row < n ? (FT)mdiag[row] : (FT)0;
    }
    return tid < 32 ? dv[I * 16 + tid - 16] : (FT)0;
  };
  FT prer = ldrow(0);
  for (int I = 0; I < nrb; ++I) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NSTG; ++s) stg[s * 256 + tid] = pre[s];
    if (tid < 32) stgr[tid] = prer;
    __syncthreads();
    if (I + 1 < nrb) {
#pragma unroll
      for (int s = 0; s <= NB; ++s) pre[s] = fr[(size_t)(I + 1) * fst + s * 256 + tid];
#pragma unroll
      for (int s = 0; s < NBL; ++s) pre[NB + 1 + s] = Dfrag[((size_t)(I + 1) * NBL + s) * 256 + tid];
      prer = ldrow(I + 1);
    }
    const V4 p2 = ld4(P2, I);
    const uint32_t mask = Dmask[I];
    V4 accD = zero4;
#pragma unroll
    for (int s = 0; s < NBL; ++s)
      if ((mask >> s) & 1u) {
#pragma unroll
        for (int v = 0; v < 4; ++v) accD = mma(stg[(NB + 1 + s) * 256 + v * 64 + lane], p1w[s][v], accD);
      }
    V4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fw1 * accD[v] + fw1s * stgr[trow<FT>(v, rsub)] * p2[v];
#pragma unroll
    for (int s = 0; s < NB; ++s)
      if (I - NB + s >= 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc = mma(stg[s * 256 + v * 64 + lane], yw[s][v], acc);
      }
    V4 y = zero4;
#pragma unroll
    for (int v = 0; v < 4; ++v) y = mma(stg[NB * 256 + v * 64 + lane], acc[v], y);
    V4 z;
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = y[v] * stgr[16 + trow<FT>(v, rsub)];
    st4(Y, I, z);
#pragma unroll
    for (int s = 0; s + 1 < NB; ++s) yw[s] = yw[s + 1];
    yw[NB - 1] = y;
#pragma unroll
    for (int s = 0; s + 1 < NBL; ++s) p1w[s] = p1w[s + 1];
    p1w[NBL - 1] = ld4(P1, I + NB + 1);
  }

  // ---------------- backward sweep
  V4 xw[NB];
#pragma unroll
  for (int s = 0; s < NB; ++s) xw[s] = zero4;
  // staged blocks of row block I: slot t - 1 = block (I + t, NB - t), t = 1..NB; slot NB = L(I,I)^-1
  {
    const int I = nrb - 1;
#pragma unroll
    for (int t = 1; t <= NB; ++t)
      pre[t - 1] = (I + t < nrb) ? fr[(size_t)(I + t) * fst + (NB - t) * 256 + tid] : (FT)0;
    pre[NB] = fr[(size_t)I * fst + NB * 256 + tid];
  }
  // the solution, P1 and P2 blocks of the next (lower) row block are loaded one block ahead
  V4 zn = ld4(Y, nrb - 1), p1n = ld4(P1, nrb - 1), p2b = ld4(P2, nrb - 1);
  int trow_, tcol_;
  opos_inv<FT>(tid, trow_, tcol_);
  const int tpos = opos<FT>(tcol_, trow_);   // where this thread's element goes in the transpose
  for (int I = nrb - 1; I >= 0; --I) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s <= NB; ++s) stg[s * 256 + tpos] = pre[s];
    __syncthreads();
    if (I > 0) {
      const int In = I - 1;
#pragma unroll
      for (int t = 1; t <= NB; ++t)
        pre[t - 1] = (In + t < nrb) ? fr[(size_t)(In + t) * fst + (NB - t) * 256 + tid] : (FT)0;
      pre[NB] = fr[(size_t)In * fst + NB * 256 + tid];
    }
    V4 acc = zn;
    const V4 p1 = p1n, p2 = p2b;
    zn = ld4(Y, I - 1);
    p1n = ld4(P1, I - 1);
    p2b = ld4(P2, I - 1);
#pragma unroll
    for (int t = 1; t <= NB; ++t)
      if (I + t < nrb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc = mma(stg[(t - 1) * 256 + v * 64 + lane], xw[t - 1][v], acc);
      }
    V4 x = zero4;
#pragma unroll
    for (int v = 0; v < 4; ++v) x = mma(stg[NB * 256 + v * 64 + lane], acc[v], x);
    V4 o1, o2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (last) {
        o1[v] = x[v];
        o2[v] = (FT)P.c2 * x[v] - p1[v];
      } else {
        o1[v] = (FT)(2.0 * P.c2) * x[v] - p1[v];
        o2[v] = (FT)(2.0 * P.c0 + P.c1 * P.c2) * x[v] - (FT)P.c1 * p1[v] - p2[v];
      }
    }
    st4(P1, I, o1);
    st4(P2, I, o2);
#pragma unroll
    for (int s = NB - 1; s > 0; --s) xw[s] = xw[s - 1];
    xw[0] = x;
  }
}

__global__ void k_widen(const float *__restrict__ src, double *__restrict__ dst, size_t len) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

// ------------------------------------------------------------------------------ host helpers
template <typename T>
fse_status wupload(fse_ctx *ctx, T **dst, const std::vector<T> &src) {
  if (hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(src.size(), 1)) != hipSuccess) {
    ctx->err = "hipMalloc failed (wide path constants)";
    return FSE_E_NOMEM;
  }
  if (!src.empty()) FSE_HIP(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
  return FSE_OK;
}

fse_status walloc(fse_ctx *ctx, void **p, size_t bytes) {
  if (*p) return FSE_OK;
  if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
    ctx->err = "hipMalloc failed (wide path buffers, " + std::to_string(bytes) + " bytes)";
    return FSE_E_NOMEM;
  }
  return FSE_OK;
}

size_t factor_lds(int bw, int NB) { return sizeof(double) * ((size_t)(bw + 1) * (bw + 1) + (size_t)(NB + 2) * 256); }

WideSys wsys(const fse_ctx *ctx, int B) {
  const WideState *ws = ctx->wide;
  return WideSys{ws->rp, ws->ci, ws->Dv, ws->Kv, ws->Sv, ws->mdiag, ctx->F, ctx->f2_ptr, ctx->f2_jk,
                 ctx->f2_v, ctx->f3_ptr, ctx->f3_jkl, ctx->f3_v, ctx->n, ws->nnz, ctx->e, ctx->d,
                 ctx->St, B * ctx->St, ctx->Wmax};
}

TrajParams wparams(const fse_ctx *ctx, int B) {
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

// S band, S on the pattern, LDL^T of S and the dense S^-1 for every point of the call
fse_status wide_point_setup(fse_ctx *ctx, int B) {
  WideState *ws = ctx->wide;
  const int n = ctx->n, bw = ctx->bw;
  const size_t nb = (size_t)n * (bw + 1);
  FSE_TRY(walloc(ctx, (void **)&ws->Sv, sizeof(double) * ctx->Bmax * ws->nnz));
  FSE_TRY(walloc(ctx, (void **)&ws->Sband, sizeof(double) * ctx->Bmax * nb));
  FSE_TRY(walloc(ctx, (void **)&ws->Sfac, sizeof(double) * nb));
  FSE_TRY(walloc(ctx, (void **)&ws->Sinv, sizeof(double) * ctx->Bmax * (size_t)n * n));
  const TrajParams P = wparams(ctx, B);
  hipLaunchKernelGGL(k_wide_sband, dim3(256, B), dim3(256), 0, ctx->stream, ctx->Mb, ctx->Db, ctx->Kb,
                     ctx->omega_d, ctx->d, n, bw, P.c0, P.c2, ws->Sband, ws->Mv, ws->Dv, ws->Kv, ws->nnz, ws->Sv);
  FSE_HIP(hipGetLastError());
  const size_t lds = factor_lds(bw, ws->NB);
  for (int b = 0; b < B; ++b) {
    hipLaunchKernelGGL((k_wide_factor<0, double>), dim3(1), dim3(kFacThreads), lds, ctx->stream,
                       ws->Sband + b * nb, nb, n, bw, ws->NB, ws->nrb, ws->Sfac, (double *)nullptr,
                       (double *)nullptr, ctx->status_d);
    hipLaunchKernelGGL(k_wide_sinv, dim3((n + 63) / 64), dim3(64), 0, ctx->stream, ws->Sfac, n, bw,
                       ws->Sinv + (size_t)b * n * n);
  }
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status wide_state_pass(fse_ctx *ctx, int B, int budget) {
  WideState *ws = ctx->wide;
  const int n = ctx->n, W = B * ctx->St, ld = ctx->Wmax;
  const TrajParams P = wparams(ctx, B);
  const WideSys sy = wsys(ctx, B);
  const dim3 g2((W + 63) / 64, n);
  hipLaunchKernelGGL(k_reset_status_wide, dim3(1), dim3(64), 0, ctx->stream, ctx->status_d, ws->ctl);
  hipLaunchKernelGGL(k_wide_init, g2, dim3(64), 0, ctx->stream, sy, ctx->omega_d, ctx->sidx_d, ctx->Sdim_d,
                     P.phib, ctx->qhist, ctx->u0, ws->u, ws->a);
  const int ntile_pt = (ctx->St + 15) / 16;
  const dim3 gc((ws->nrb + 3) / 4, B * ntile_pt);
  const dim3 gr(ws->nrb, (W + kLanes - 1) / kLanes);
  const size_t rl = sizeof(double) * (size_t)ws->span_r * kLanes;
  for (int k = 0; k < P.S1; ++k) {
    const double *q = ctx->qhist + (size_t)k * n * ld;
    double *qn = ctx->qhist + (size_t)(k + 1) * n * ld;
    hipLaunchKernelGGL(k_wide_predict, g2, dim3(64), 0, ctx->stream, sy, P, k, ctx->omega_d, ctx->sidx_d,
                       ctx->Sdim_d, q, ws->u, ws->a, ws->bk, ws->qh, ws->acc, ws->conv, ws->ndprev, ws->ctl);
    for (int it = 0; it < budget; ++it) {
      hipLaunchKernelGGL(k_wide_resid, gr, dim3(kResThreads), rl, ctx->stream, sy, ws->rlo, ws->span_r, ws->qh,
                         ws->bk, ws->r, ws->conv, ws->ctl);
      hipLaunchKernelGGL(k_wide_chord, gc, dim3(kChordThreads), 0, ctx->stream, n, W, ctx->St, ld, ntile_pt, ws->Sinv,
                         ws->r, ws->qh, ws->acc, ws->conv, ws->ndprev, ws->ctl, it, budget - 1,
                         (int)(budget >= ctx->maxit), k, ctx->tol, ctx->status_d);
    }
    hipLaunchKernelGGL(k_wide_update, g2, dim3(64), 0, ctx->stream, n, W, ld, P, ws->qh, q, qn, ws->u, ws->a,
                       (int)(k == P.S1 - 1), ctx->zTw, ctx->status_d);
  }
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

}  // namespace


fse_status wide_prepare(fse_ctx *ctx, const std::vector<double> &Mb, const std::vector<double> &Db,
                        const std::vector<double> &Kb, const std::vector<int32_t> &p2,
                        const std::vector<int32_t> &jk, const std::vector<int32_t> &p3,
                        const std::vector<int32_t> &jkl, const std::vector<int32_t> &ktp,
                        const std::vector<int32_t> &kti) {
  const int n = ctx->n, bw = ctx->bw, W2 = 2 * bw + 1, P = bw + 1;
  if (ctx->has_vel || bw < 1 || (bw + 15) / 16 > kMaxNB) return FSE_OK;
  // lumped (diagonal, positive) mass only
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < W2; ++t) {
      const double v = Mb[(size_t)i * W2 + t];
      if (t == bw ? !(v > 0.0) : v != 0.0) return FSE_OK;
    }
  auto ws = new WideState();
  ws->n = n;
  ws->bw = bw;
  ws->NB = (bw + 15) / 16;
  ws->nrb = (n + 15) / 16;
  const int NB = ws->NB, nrb = ws->nrb, NBL = 2 * NB + 1;
  // CSR pattern of M + D + K and the values of each on it
  std::vector<int32_t> rp(n + 1, 0), ci;
  std::vector<double> Mv, Dv, Kv, mdiag(n);
  for (int i = 0; i < n; ++i) {
    for (int t = 0; t < W2; ++t) {
      const int j = i - bw + t;
      if (j < 0 || j >= n) continue;
      const size_t e = (size_t)i * W2 + t;
      if (Mb[e] == 0.0 && Db[e] == 0.0 && Kb[e] == 0.0) continue;
      ci.push_back(j);
      Mv.push_back(Mb[e]);
      Dv.push_back(Db[e]);
      Kv.push_back(Kb[e]);
    }
    rp[i + 1] = (int32_t)ci.size();
    mdiag[i] = Mb[(size_t)i * W2 + bw];
  }
  ws->nnz = (int)ci.size();
  // lower band of K, column-major
  std::vector<double> Kl((size_t)n * P, 0.0);
  for (int m = 0; m < n; ++m)
    for (int r = 0; r <= bw && m + r < n; ++r) Kl[(size_t)m * P + r] = Kb[(size_t)(m + r) * W2 + (bw - r)];
  // D blocks around the diagonal in forward-fragment order, and their nonzero mask
  std::vector<double> Df((size_t)nrb * NBL * 256, 0.0);
  std::vector<float> Df32((size_t)nrb * NBL * 256, 0.0f);
  std::vector<uint32_t> Dm(nrb, 0u);
  for (int I = 0; I < nrb; ++I)
    for (int s = 0; s < NBL; ++s) {
      const int J = I - NB + s;
      if (J < 0 || J >= nrb) continue;
      for (int row = 0; row < 16; ++row)
        for (int col = 0; col < 16; ++col) {
          const int i = 16 * I + row, j = 16 * J + col;
          if (i >= n || j >= n || std::abs(i - j) > bw) continue;
          const double v = Db[(size_t)i * W2 + (j - i + bw)];
          if (v == 0.0) continue;
          Df[((size_t)I * NBL + s) * 256 + opos<double>(row, col)] = v;
          Df32[((size_t)I * NBL + s) * 256 + opos<float>(row, col)] = (float)v;
          Dm[I] |= 1u << s;
        }
    }
  // rows of q staged by the residual blocks (matrix pattern and tensor indices of their rows)
  // and by the tangent blocks (indices of the contribution lists of their band columns)
  std::vector<int32_t> rlo(nrb), tlo(nrb);
  int span_r = 1, span_t = 1;
  for (int I = 0; I < nrb; ++I) {
    int lo = INT_MAX, hi = INT_MIN;
    for (int i = 16 * I; i < std::min(n, 16 * I + 16); ++i) {
      lo = std::min(lo, i);
      hi = std::max(hi, i);
      for (int p = rp[i]; p < rp[i + 1]; ++p) lo = std::min(lo, ci[p]), hi = std::max(hi, ci[p]);
      for (int p = p2[i]; p < p2[i + 1]; ++p)
        for (int a = 0; a < 2; ++a) lo = std::min(lo, jk[2 * p + a]), hi = std::max(hi, jk[2 * p + a]);
      for (int p = p3[i]; p < p3[i + 1]; ++p)
        for (int a = 0; a < 3; ++a) lo = std::min(lo, jkl[3 * p + a]), hi = std::max(hi, jkl[3 * p + a]);
    }
    rlo[I] = lo;
    span_r = std::max(span_r, hi - lo + 1);
    lo = INT_MAX;
    hi = INT_MIN;
    for (int m = 16 * I; m < std::min(n, 16 * I + 16); ++m)
      for (int r = 0; r <= bw; ++r) {
        const size_t pos = (size_t)m * P + r;
        for (int p = ktp[pos]; p < ktp[pos + 1]; ++p)
          for (int a = 0; a < 2; ++a) {
            const int x = kti[2 * p + a];
            if (x >= 0) lo = std::min(lo, x), hi = std::max(hi, x);
          }
      }
    if (lo > hi) lo = hi = 16 * I;
    tlo[I] = lo;
    span_t = std::max(span_t, hi - lo + 1);
  }
  ws->span_r = span_r;
  ws->span_t = span_t;
  const size_t tile_lds = sizeof(double) * 64 * 65;
  if ((size_t)span_r * kLanes * sizeof(double) > (size_t)kStageLds ||
      (size_t)span_t * kLanes * sizeof(double) + tile_lds > (size_t)kStageLds + 10 * 1024 ||
      factor_lds(bw, NB) > 160 * 1024) {
    delete ws;  // the staged rows do not fit in LDS: the generic kernels serve this system
    return FSE_OK;
  }
  ctx->wide = ws;
  FSE_TRY(wupload(ctx, &ws->rp, rp));
  FSE_TRY(wupload(ctx, &ws->ci, ci));
  FSE_TRY(wupload(ctx, &ws->Mv, Mv));
  FSE_TRY(wupload(ctx, &ws->Dv, Dv));
  FSE_TRY(wupload(ctx, &ws->Kv, Kv));
  FSE_TRY(wupload(ctx, &ws->mdiag, mdiag));
  FSE_TRY(wupload(ctx, &ws->Kband, Kl));
  FSE_TRY(wupload(ctx, &ws->Dfrag, Df));
  FSE_TRY(wupload(ctx, &ws->Dfrag32, Df32));
  FSE_TRY(wupload(ctx, &ws->Dmask, Dm));
  FSE_TRY(wupload(ctx, &ws->rlo, rlo));
  FSE_TRY(wupload(ctx, &ws->tlo, tlo));
  return FSE_OK;
}

bool wide_eligible(const fse_ctx *ctx) {
  if (!ctx->wide || ctx->has_vel || ctx->ncon != 0 || ctx->nm_beta != 0.25 || ctx->nm_gamma != 0.5) return false;
  if (!ctx->use_wide) return false;
  return ctx->wide_forced || !fused_eligible(ctx);
}

fse_status launch_wide_state(fse_ctx *ctx, int B) {
  WideState *ws = ctx->wide;
  const size_t nW = (size_t)ctx->n * ctx->Wmax;
  FSE_TRY(walloc(ctx, (void **)&ws->u, sizeof(double) * nW));
  FSE_TRY(walloc(ctx, (void **)&ws->a, sizeof(double) * nW));
  FSE_TRY(walloc(ctx, (void **)&ws->bk, sizeof(double) * nW));
  FSE_TRY(walloc(ctx, (void **)&ws->qh, sizeof(double) * nW));
  FSE_TRY(walloc(ctx, (void **)&ws->r, sizeof(double) * nW));
  FSE_TRY(walloc(ctx, (void **)&ws->acc, sizeof(unsigned long long) * 4 * ctx->Wmax));
  FSE_TRY(walloc(ctx, (void **)&ws->conv, sizeof(int32_t) * ctx->Wmax));
  FSE_TRY(walloc(ctx, (void **)&ws->ndprev, sizeof(double) * ctx->Wmax));
  FSE_TRY(walloc(ctx, (void **)&ws->ctl, sizeof(int32_t) * 4));
  FSE_TRY(wide_point_setup(ctx, B));
  // chord iterations launched per step: adapted to the last call; if a trajectory needs more,
  // the pass is repeated once with the full budget (step_maxit), after which it is NOCONV
  int budget = std::min(std::max(ws->budget, 2), ctx->maxit);
  for (int attempt = 0; attempt < 2; ++attempt) {
    FSE_TRY(wide_state_pass(ctx, B, budget));
    int32_t hit = 0;
    DevStatus st;
    FSE_HIP(hipMemcpyAsync(&hit, ws->ctl + 2, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    FSE_HIP(hipMemcpyAsync(&st, ctx->status_d, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
    FSE_HIP(hipStreamSynchronize(ctx->stream));
    if (!hit || budget >= ctx->maxit) {
      if (!hit) ws->budget = std::min(ctx->maxit, st.max_iters + 2);
      break;
    }
    budget = ctx->maxit;
  }
  return FSE_OK;
}

fse_status launch_wide_sens(fse_ctx *ctx, int B, double *Phi) {
  WideState *ws = ctx->wide;
  const int n = ctx->n, bw = ctx->bw, NB = ws->NB, nrb = ws->nrb, W = B * ctx->St, ld = ctx->Wmax;
  const size_t nb = (size_t)n * (bw + 1), n2 = 2 * (size_t)n;
  const bool f32 = ctx->prec == FSE_PREC_MIXED_FP32;
  const size_t fs = f32 ? sizeof(float) : sizeof(double);
  const size_t tb_el = (size_t)ctx->Wmax * nb, fr_el = (size_t)ctx->Wmax * nrb * (NB + 1) * 256,
               dv_el = (size_t)ctx->Wmax * nrb * 16;
  FSE_TRY(walloc(ctx, (void **)&ws->Tband, sizeof(double) * 2 * tb_el));
  if (ws->frag && ws->frag_bytes != fs) {
    (void)hipFree(ws->frag);
    (void)hipFree(ws->dinv);
    (void)hipFree(ws->Ysc);
    ws->frag = ws->dinv = ws->Ysc = nullptr;
  }
  ws->frag_bytes = fs;
  FSE_TRY(walloc(ctx, &ws->frag, fs * 2 * fr_el));
  FSE_TRY(walloc(ctx, &ws->dinv, fs * 2 * dv_el));
  FSE_TRY(walloc(ctx, &ws->Ysc, fs * ctx->Wmax * n * n2));
  if (f32) FSE_TRY(walloc(ctx, (void **)&ws->P32, sizeof(float) * ctx->Wmax * n2 * n2));
  if (!ws->side) {
    FSE_HIP(hipStreamCreateWithFlags(&ws->side, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
      FSE_HIP(hipEventCreateWithFlags(&ws->ev_fac[b], hipEventDisableTiming));
      FSE_HIP(hipEventCreateWithFlags(&ws->ev_sw[b], hipEventDisableTiming));
    }
    FSE_HIP(hipEventCreateWithFlags(&ws->ev_go, hipEventDisableTiming));
  }
  const TrajParams P = wparams(ctx, B);
  while ((int)ws->ev_k.size() < 2 * P.S1) {
    hipEvent_t e;
    FSE_HIP(hipEventCreate(&e));
    ws->ev_k.push_back(e);
  }
  ws->ev_used = 0;
  const dim3 gt(nrb, (W + kLanes - 1) / kLanes);
  const size_t tl = sizeof(double) * ((size_t)ws->span_t * kLanes + 64 * 65);
  const size_t fl = factor_lds(bw, NB);
  // A_0 from K + K_t(q_0), then the seeds P1_0, P2_0
  hipLaunchKernelGGL(k_wide_tangent, gt, dim3(256), tl, ctx->stream, n, bw, W, ctx->St, ld, ws->tlo, ws->span_t,
                     ctx->qhist, ctx->kt_ptr, ctx->kt_idx, ctx->kt_c, ws->Kband, (size_t)0, ws->Tband);
  if (f32)
    hipLaunchKernelGGL(k_wide_sens0<float>, dim3(2 * n, W), dim3(256), 0, ctx->stream, n, bw, W, ctx->St, ctx->d,
                       P, ctx->omega_d, ws->Tband, ctx->Db, ws->mdiag, ws->P32);
  else
    hipLaunchKernelGGL(k_wide_sens0<double>, dim3(2 * n, W), dim3(256), 0, ctx->stream, n, bw, W, ctx->St, ctx->d,
                       P, ctx->omega_d, ws->Tband, ctx->Db, ws->mdiag, Phi);
  FSE_HIP(hipGetLastError());
  // the side stream starts after everything enqueued so far (states, seeds)
  FSE_HIP(hipEventRecord(ws->ev_go, ctx->stream));
  FSE_HIP(hipStreamWaitEvent(ws->side, ws->ev_go, 0));
  const int ntiles = (int)((n2 + 15) / 16), ncg = (ntiles + 3) / 4;
  const bool exact = n % 16 == 0;
  const int per_xcd = (W * ncg + 7) / 8;
  const dim3 gs(8 * per_xcd);
  for (int k = 0; k < P.S1; ++k) {
    const int bf = k & 1;
    double *Tb = ws->Tband + bf * tb_el;
    void *fr = (char *)ws->frag + fs * bf * fr_el;
    void *dv = (char *)ws->dinv + fs * bf * dv_el;
    // side stream: T_{k+1} and its factor, once the sweep two steps back has released the buffer
    if (k >= 2) FSE_HIP(hipStreamWaitEvent(ws->side, ws->ev_sw[bf], 0));
    const double *q = ctx->qhist + (size_t)(k + 1) * n * ld;
    hipLaunchKernelGGL(k_wide_tangent, gt, dim3(256), tl, ws->side, n, bw, W, ctx->St, ld, ws->tlo,
                       ws->span_t, q, ctx->kt_ptr, ctx->kt_idx, ctx->kt_c, ws->Sband, nb, Tb);
    if (f32)
      hipLaunchKernelGGL((k_wide_factor<1, float>), dim3(W), dim3(kFacThreads), fl, ws->side, Tb, nb, n,
                         bw, NB, nrb, (double *)nullptr, (float *)fr, (float *)dv, ctx->status_d);
    else
      hipLaunchKernelGGL((k_wide_factor<1, double>), dim3(W), dim3(kFacThreads), fl, ws->side, Tb, nb, n,
                         bw, NB, nrb, (double *)nullptr, (double *)fr, (double *)dv, ctx->status_d);
    FSE_HIP(hipEventRecord(ws->ev_fac[bf], ws->side));
    // context stream: the sweep of step k
    FSE_HIP(hipStreamWaitEvent(ctx->stream, ws->ev_fac[bf], 0));
    const int last = k == P.S1 - 1;
    FSE_HIP(hipEventRecord(ws->ev_k[2 * k], ctx->stream));
    if (f32) {
#define WIDE_SWEEP32(NBV)                                                                                      \
  if (exact)                                                                                                   \
    hipLaunchKernelGGL((k_wide_sweep<NBV, float, true>), gs, dim3(256), 0, ctx->stream, n, W, ctx->St, ctx->d,   \
                       nrb, ncg, per_xcd, ctx->omega_d, P, ws->mdiag, ws->Dfrag32, ws->Dmask, (const float *)fr, \
                       (const float *)dv, ws->P32, (float *)ws->Ysc, last);                                     \
  else                                                                                                         \
    hipLaunchKernelGGL((k_wide_sweep<NBV, float, false>), gs, dim3(256), 0, ctx->stream, n, W, ctx->St, ctx->d,  \
                       nrb, ncg, per_xcd, ctx->omega_d, P, ws->mdiag, ws->Dfrag32, ws->Dmask, (const float *)fr, \
                       (const float *)dv, ws->P32, (float *)ws->Ysc, last)
      switch (NB) {
        case 1: WIDE_SWEEP32(1); break;
        case 2: WIDE_SWEEP32(2); break;
        case 3: WIDE_SWEEP32(3); break;
        case 4: WIDE_SWEEP32(4); break;
        case 5: WIDE_SWEEP32(5); break;
        default: WIDE_SWEEP32(6); break;
      }
#undef WIDE_SWEEP32
    } else {
#define WIDE_SWEEP64(NBV)                                                                                       \
  if (exact)                                                                                                    \
    hipLaunchKernelGGL((k_wide_sweep<NBV, double, true>), gs, dim3(256), 0, ctx->stream, n, W, ctx->St, ctx->d,   \
                       nrb, ncg, per_xcd, ctx->omega_d, P, ws->mdiag, ws->Dfrag, ws->Dmask, (const double *)fr,   \
                       (const double *)dv, Phi, (double *)ws->Ysc, last);                                        \
  else                                                                                                          \
    hipLaunchKernelGGL((k_wide_sweep<NBV, double, false>), gs, dim3(256), 0, ctx->stream, n, W, ctx->St, ctx->d,  \
                       nrb, ncg, per_xcd, ctx->omega_d, P, ws->mdiag, ws->Dfrag, ws->Dmask, (const double *)fr,   \
                       (const double *)dv, Phi, (double *)ws->Ysc, last)
      switch (NB) {
        case 1: WIDE_SWEEP64(1); break;
        case 2: WIDE_SWEEP64(2); break;
        case 3: WIDE_SWEEP64(3); break;
        case 4: WIDE_SWEEP64(4); break;
        case 5: WIDE_SWEEP64(5); break;
        default: WIDE_SWEEP64(6); break;
      }
#undef WIDE_SWEEP64
    }
    FSE_HIP(hipEventRecord(ws->ev_k[2 * k + 1], ctx->stream));
    FSE_HIP(hipEventRecord(ws->ev_sw[bf], ctx->stream));
  }
  ws->ev_used = P.S1;
  if (f32)
    hipLaunchKernelGGL(k_widen, dim3(4096), dim3(256), 0, ctx->stream, ws->P32, Phi, (size_t)W * n2 * n2);
  ctx->last_sens_launches = 3 * P.S1 + 2;
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status wide_sweep_timing(fse_ctx *ctx, double *ms_total, int *launches) {
  WideState *ws = ctx->wide;
  *ms_total = 0.0;
  *launches = 0;
  if (!ws || ws->ev_used == 0) return FSE_OK;
  for (int k = 0; k < ws->ev_used; ++k) {
    float ms = 0.0f;
    FSE_HIP(hipEventElapsedTime(&ms, ws->ev_k[2 * k], ws->ev_k[2 * k + 1]));
    *ms_total += ms;
  }
  *launches = ws->ev_used;
  return FSE_OK;
}

void wide_free(fse_ctx *ctx) {
  WideState *ws = ctx->wide;
  if (!ws) return;
  void *ptrs[] = {ws->rp, ws->ci, ws->Mv, ws->Dv, ws->Kv, ws->mdiag, ws->Dfrag, ws->Dfrag32, ws->Dmask,
                  ws->rlo, ws->tlo, ws->Kband, ws->Sv, ws->Sband, ws->Sfac, ws->Sinv, ws->u, ws->a, ws->bk,
                  ws->qh, ws->r, ws->acc, ws->conv, ws->ndprev, ws->ctl, ws->Tband, ws->frag, ws->dinv,
                  ws->Ysc, ws->P32};
  if (ws->side) {
    (void)hipStreamSynchronize(ws->side);
    (void)hipStreamDestroy(ws->side);
    for (int b = 0; b < 2; ++b) {
      (void)hipEventDestroy(ws->ev_fac[b]);
      (void)hipEventDestroy(ws->ev_sw[b]);
    }
    (void)hipEventDestroy(ws->ev_go);
  }
  for (hipEvent_t e : ws->ev_k) (void)hipEventDestroy(e);
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete ws;
  ctx->wide = nullptr;
}
