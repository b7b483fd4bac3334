// Dense FP64 linear algebra for the shooting Newton step (Sec. 3.3 step 6) and
// the Lyapunov exponents (App. F) on gfx950.
#include <cmath>
#include <vector>

#include "fse_internal.h"

namespace {

// ---------------------------------------------------------------- LU with partial pivoting
// The Jacobian arrives row-major (J[i][j] at i*N + j).  The factorisation works on
// B = J^T read column-major (B(i, j) at j*N + i), so a column of B is contiguous and
// pivot searches and rank-1 updates are coalesced:  Pi B = L U with unit lower L and
// row interchanges Pi = S_{N-1} ... S_0 (S_k swaps k and piv[k]).  Then
// J = U^T L^T Pi, and J x = r is solved as U^T v = r, L^T w = v, x = Pi^T w.
// Right-looking blocked algorithm with recursively split panels.

constexpr int kLuLeaf = 8;    // panel columns factored by one work-group
constexpr int kLuBlock = 64;  // outer block (also the largest TRSM triangle)

// Factor the leaf panel B[j0:N, j0:j0+nb] (nb <= kLuLeaf) with partial pivoting;
// interchanges are applied inside the panel only.
template <typename T>
__global__ __launch_bounds__(1024) void k_lu_leaf(T *__restrict__ B, int N, int j0, int nb,
                                                  int32_t *__restrict__ piv, DevStatus *st) {
  __shared__ T sv[16];
  __shared__ int si[16];
  __shared__ int piv_s;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  for (int c = 0; c < nb; ++c) {
    const int j = j0 + c;
    const T *col = B + (size_t)j * N;
    T best = T(-1);
    int bi = j;
    for (int i = j + tid; i < N; i += nt) {
      const T v = fabs(col[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const T ov = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      sv[wid] = best;
      si[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      T b = sv[0];
      int ix = si[0];
      for (int w = 1; w < (nt >> 6); ++w)
        if (sv[w] > b || (sv[w] == b && si[w] < ix)) {
          b = sv[w];
          ix = si[w];
        }
      piv_s = ix;
      piv[j] = ix;
      if (!(b > T(0)) || !isfinite(b)) atomicOr(&st->flags, (int)DEV_SINGULAR);
    }
    __syncthreads();
    const int p = piv_s;
    if (p != j && tid < nb) {
      T *cc = B + (size_t)(j0 + tid) * N;
      const T t = cc[j];
      cc[j] = cc[p];
      cc[p] = t;
    }
    __syncthreads();
    const T inv = T(1) / col[j];
    for (int i = j + 1 + tid; i < N; i += nt) {
      const T l = col[i] * inv;
      B[(size_t)j * N + i] = l;
      for (int c2 = c + 1; c2 < nb; ++c2) {
        T *cc = B + (size_t)(j0 + c2) * N;
        cc[i] -= l * cc[j];
      }
    }
    __syncthreads();
  }
}

// The same leaf with the panel held in registers: thread t owns rows j0 + t + 1024 r
// (r < RPT) of the NB columns, so each column costs one block reduction for the pivot and one
// exchange of the pivot row and row j through LDS, and the rank-1 update never leaves the
// registers.  Pivots and arithmetic are those of k_lu_leaf.  Needs N - j0 <= 1024 RPT.
template <typename T, int NB, int RPT>
__global__ __launch_bounds__(1024) void k_lu_leaf_reg(T *__restrict__ B, int N, int j0, int nb,
                                                      int32_t *__restrict__ piv, DevStatus *st) {
  constexpr int NT = 1024;
  __shared__ T sv[NT / 64];
  __shared__ int si[NT / 64];
  __shared__ T prow[NB], jrow[NB];
  __shared__ int piv_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T v[RPT][NB];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = j0 + tid + r * NT;
#pragma unroll
    for (int c = 0; c < NB; ++c) v[r][c] = (i < N && c < nb) ? B[(size_t)(j0 + c) * N + i] : T(0);
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= nb) break;
    const int j = j0 + c;
    T best = T(-1);
    int bi = j;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = j0 + tid + r * NT;
      const T a = fabs(v[r][c]);
      if (i >= j && i < N && a > best) {
        best = a;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const T ov = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      sv[wid] = best;
      si[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      T b = sv[0];
      int ix = si[0];
      for (int w = 1; w < NT / 64; ++w)
        if (sv[w] > b || (sv[w] == b && si[w] < ix)) {
          b = sv[w];
          ix = si[w];
        }
      piv_s = ix;
      piv[j] = ix;
      if (!(b > T(0)) || !isfinite(b)) atomicOr(&st->flags, (int)DEV_SINGULAR);
    }
    __syncthreads();
    const int p = piv_s;
    const int tp = (p - j0) % NT, rp = (p - j0) / NT;  // owner of row p; row j is thread c, slot 0
    if (tid == tp) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == rp) {
#pragma unroll
          for (int c2 = 0; c2 < NB; ++c2) prow[c2] = v[r][c2];
        }
    }
    if (tid == c) {
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) jrow[c2] = v[0][c2];
    }
    __syncthreads();
    if (p != j) {
      if (tid == c) {
#pragma unroll
        for (int c2 = 0; c2 < NB; ++c2) v[0][c2] = prow[c2];
      }
      if (tid == tp) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (r == rp) {
#pragma unroll
            for (int c2 = 0; c2 < NB; ++c2) v[r][c2] = jrow[c2];
          }
      }
    }
    const T inv = T(1) / prow[c];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = j0 + tid + r * NT;
      if (i > j && i < N) {
        const T l = v[r][c] * inv;
        v[r][c] = l;
#pragma unroll
        for (int c2 = c + 1; c2 < NB; ++c2) v[r][c2] -= l * prow[c2];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = j0 + tid + r * NT;
    if (i >= N) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) B[(size_t)(j0 + c) * N + i] = v[r][c];
  }
}

// Interchanges piv[k0..k1) applied in order to the columns [c0, c1) of B.
template <typename T>
__global__ void k_lu_swap(T *__restrict__ B, int N, int c0, int c1, int k0, int k1,
                          const int32_t *__restrict__ piv) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  T *cc = B + (size_t)c * N;
  for (int k = k0; k < k1; ++k) {
    const int p = piv[k];
    if (p != k) {
      const T t = cc[k];
      cc[k] = cc[p];
      cc[p] = t;
    }
  }
}

// B[j0:j0+nb, c0:c0+nc] <- L11^-1 B[j0:j0+nb, c0:c0+nc], L11 the unit lower triangle of
// B[j0:j0+nb, j0:j0+nb] (nb <= 64) staged in LDS.  One wave per column, lane r holds row r.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_trsm(T *__restrict__ B, int N, int j0, int nb, int c0,
                                                 int nc) {
  __shared__ T L[kLuBlock][kLuBlock + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int r = e % nb, c = e / nb;
    L[r][c] = B[(size_t)(j0 + c) * N + j0 + r];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int col = c0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= c0 + nc) return;
  T *cc = B + (size_t)col * N + j0;
  T x = lane < nb ? cc[lane] : T(0);
  for (int r = 0; r < nb - 1; ++r) {
    const T xr = __shfl(x, r);
    if (lane > r) x -= L[lane][r] * xr;
  }
  if (lane < nb) cc[lane] = x;
}

// C -= A Bm on column-major sub-blocks of B: C = B[r0:r0+m, c0:c0+n], A = B[r0:r0+m, k0:k0+kk],
// Bm = B[k0:k0+kk, c0:c0+n].  64 x 64 tiles, 16-deep k slices staged in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_gemm(T *__restrict__ B, int N, int r0, int m, int c0,
                                                 int n, int k0, int kk) {
  __shared__ T As[16][68];
  __shared__ T Bs[16][68];
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  const int i0 = r0 + blockIdx.x * 64, jb = c0 + blockIdx.y * 64;
  T acc[4][4] = {};
  for (int ks = 0; ks < kk; ks += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int i = e & 63, k = e >> 6;
      const int gi = i0 + i, gk = k0 + ks + k;
      As[k][i] = (gi < r0 + m && ks + k < kk) ? B[(size_t)gk * N + gi] : T(0);
      const int k2 = e & 15, j = e >> 4;
      const int gj = jb + j, gk2 = k0 + ks + k2;
      Bs[k2][j] = (gj < c0 + n && ks + k2 < kk) ? B[(size_t)gj * N + gk2] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      T a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[k][tr + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bs[k][tc + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gj = jb + tc + 16 * v;
    if (gj >= c0 + n) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gi = i0 + tr + 16 * u;
      if (gi < r0 + m) B[(size_t)gj * N + gi] -= acc[u][v];
    }
  }
}

// Blocked triangular solves with the factors of B (row i of U^T and of L^T is contiguous:
// memory row i).  For the rows [r0, r0+nb) the already solved columns [c0, c1) contribute
// M[r0:r0+nb, cols] x[cols]; they are split into chunks of kGemvChunk columns, one work-group per
// 4 rows and chunk (one wave per row), each writing its partial sums, which the diagonal kernel
// then adds in chunk order.  The solve kernels take a batch of independent systems of one size,
// system z at A + z sA, its vectors at x + z sx, its pivots at piv + z sp and its partial sums at
// part + z spp.
constexpr int kGemvChunk = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_lu_gemv(const T *__restrict__ A, int N, int r0, int nb,
                                                 int c0, int c1, const T *__restrict__ x,
                                                 T *__restrict__ part, size_t sA, size_t sx, size_t spp) {
  A += blockIdx.z * sA;
  x += blockIdx.z * sx;
  part += blockIdx.z * spp;
  const int lane = threadIdx.x & 63;
  const int rr = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (rr >= nb) return;
  const int ch = blockIdx.y;
  const int ca = c0 + ch * kGemvChunk, cb = min(c1, ca + kGemvChunk);
  const T *row = A + (size_t)(r0 + rr) * N;
  T s = T(0);
  for (int c = ca + lane; c < cb; c += 64) s += row[c] * x[c];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) part[(size_t)ch * 64 + rr] = s;
}

// Diagonal block of the substitution, one wave: forward (upper = false: U^T with its
// diagonal) or backward (upper = true: unit L^T) over rows [r0, r0+nb), nb <= 64, after the
// nch partial sums of the solved columns are subtracted.  The block is staged in LDS first
// (coalesced rows), so the dependent chain of the substitution runs at LDS latency.
template <typename T>
__global__ __launch_bounds__(64) void k_lu_diag(const T *__restrict__ A, int N, int r0, int nb,
                                                bool upper, T *__restrict__ y, const T *__restrict__ part,
                                                int nch, size_t sA, size_t sx, size_t spp) {
  __shared__ T Ds[64][65];
  A += blockIdx.x * sA;
  y += blockIdx.x * sx;
  part += blockIdx.x * spp;
  const int lane = threadIdx.x;
  for (int row = 0; row < nb; ++row) Ds[row][lane] = lane < nb ? A[(size_t)(r0 + row) * N + r0 + lane] : T(0);
  T x = lane < nb ? y[r0 + lane] : T(0);
  if (lane < nb)
    for (int ch = 0; ch < nch; ++ch) x -= part[(size_t)ch * 64 + lane];
  __syncthreads();
  if (!upper) {
    for (int r = 0; r < nb; ++r) {
      const T xr = __shfl(x, r) / Ds[r][r];
      if (lane == r) x = xr;
      // rows below: memory row (r0+lane), column (r0+r)
      if (lane > r && lane < nb) x -= Ds[lane][r] * xr;
    }
  } else {
    for (int r = nb - 1; r >= 0; --r) {
      const T xr = __shfl(x, r);
      if (lane < r) x -= Ds[lane][r] * xr;
    }
  }
  if (lane < nb) y[r0 + lane] = x;
}

// x = Pi^T w: interchanges applied in reverse order (one thread).
// x <- Pi^T x: the interchanges in reverse order.  Vectors of up to kUnpermLds entries are
// staged in LDS so the serial chain of swaps runs at LDS latency.
constexpr int kUnpermLds = 16384;

template <typename T>
__global__ __launch_bounds__(1024) void k_lu_unpermute(T *__restrict__ x, int N,
                                                       const int32_t *__restrict__ piv, size_t sx, size_t sp) {
  extern __shared__ __align__(16) unsigned char xs_raw[];
  T *xs = reinterpret_cast<T *>(xs_raw);
  x += blockIdx.x * sx;
  piv += blockIdx.x * sp;
  if (N <= kUnpermLds) {
    // the two memories get separate code so that no pointer may point to either
    for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = x[i];
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = N - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k) {
          const T t = xs[k];
          xs[k] = xs[p];
          xs[p] = t;
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) x[i] = xs[i];
  } else if (threadIdx.x == 0) {
    for (int k = N - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k) {
        const T t = x[k];
        x[k] = x[p];
        x[p] = t;
      }
    }
  }
}

__global__ void k_axpby(int N, double a, const double *__restrict__ x, double b, const double *__restrict__ z,
                        double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = a * x[i] + b * z[i];
}

__global__ void k_lincomb(int N, const double *__restrict__ x, double alpha, const double *__restrict__ d,
                          double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = x[i] + alpha * d[i];
}

__global__ void k_axpy(int N, double alpha, const double *__restrict__ x, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] += alpha * x[i];
}

// ---------------------------------------------------------------- Lyapunov exponents
// Psihat[l][ij] = sum_s Gamma^-1[l][s] Psi_s[ij], Psi_s = diag(I, w I) Phi_s diag(I, I/w)  (Eq. F3)
__global__ void k_psi_hat(const double *__restrict__ Phi, const double *__restrict__ Gi, int n, int U,
                          int St, double w1, double *__restrict__ Ph) {
  const size_t n2 = 2 * (size_t)n, NIJ = n2 * n2;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NIJ * U) return;
  const size_t ij = idx % NIJ;
  const int l = (int)(idx / NIJ);
  const int i = (int)(ij / n2), j = (int)(ij % n2);
  const double sc = (i >= n ? w1 : 1.0) / (j >= n ? w1 : 1.0);
  double v = 0.0;
  for (int s = 0; s < St; ++s) v += Gi[(size_t)l * St + s] * Phi[(size_t)s * NIJ + ij];
  Ph[idx] = v * sc;
}

// Psi_i[ij] = sum_l H_i[l] Psihat[l][ij]
__global__ void k_psi_interp(const double *__restrict__ Ph, const double *__restrict__ H, int U,
                             size_t NIJ, double *__restrict__ Psi) {
  const size_t ij = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ij >= NIJ) return;
  double v = 0.0;
  for (int l = 0; l < U; ++l) v += H[l] * Ph[(size_t)l * NIJ + ij];
  Psi[ij] = v;
}

// C = A B for m x m row-major matrices, 64 x 64 tiles.
__global__ __launch_bounds__(256) void k_gemm_sq(const double *__restrict__ A, const double *__restrict__ B,
                                                 int m, double *__restrict__ C) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < m; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, cc = e % 64;
      As[kk][cc] = (r0 + cc < m && k0 + kk < m) ? A[(size_t)(r0 + cc) * m + k0 + kk] : 0.0;
      Bs[kk][cc] = (k0 + kk < m && c0 + cc < m) ? B[(size_t)(k0 + kk) * m + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + ty * 4 + i, c = c0 + tx * 4 + j;
      if (r < m && c < m) C[(size_t)r * m + c] = acc[i][j];
    }
}

// Householder QR of the m x m row-major Y in place (one block); accumulates
// log|R_hh| into acc and writes the explicit orthogonal factor into Q.
__global__ __launch_bounds__(1024) void k_householder(double *__restrict__ Y, int m, double *__restrict__ Q,
                                                      double *__restrict__ beta, double *__restrict__ acc,
                                                      DevStatus *st) {
  __shared__ double red[16];
  __shared__ double sh_alpha, sh_beta;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  for (int j = 0; j < m; ++j) {
    // sigma = ||Y[j+1:, j]||^2
    double s = 0.0;
    for (int r = j + 1 + tid; r < m; r += nt) {
      const double v = Y[(size_t)r * m + j];
      s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (tid == 0) {
      double sig = 0.0;
      for (int w = 0; w < (nt >> 6); ++w) sig += red[w];
      const double x0 = Y[(size_t)j * m + j];
      const double nrm = sqrt(x0 * x0 + sig);
      // v = x - alpha e1 with alpha = -sign(x0) ||x||, stored with v0 = x0 - alpha in place
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vtv = v0 * v0 + sig;
      sh_alpha = alpha;
      sh_beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
      Y[(size_t)j * m + j] = v0;
      beta[j] = sh_beta;
      if (!(nrm > 0.0) || !isfinite(nrm)) atomicOr(&st->flags, (int)DEV_SINGULAR);
      acc[j] += log(fabs(alpha));
    }
    __syncthreads();
    const double bj = sh_beta;
    // apply H = I - beta v v^T to columns j+1..m-1
    for (int c = j + 1 + tid; c < m; c += nt) {
      double w = 0.0;
      for (int r = j; r < m; ++r) w += Y[(size_t)r * m + j] * Y[(size_t)r * m + c];
      w *= bj;
      for (int r = j; r < m; ++r) Y[(size_t)r * m + c] -= w * Y[(size_t)r * m + j];
    }
    __syncthreads();
  }
  // Q = H_0 H_1 ... H_{m-1}: start from I and apply H_j from the left for j = m-1..0
  for (int e = tid; e < m * m; e += nt) Q[e] = ((e / m) == (e % m)) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = m - 1; j >= 0; --j) {
    const double bj = beta[j];
    for (int c = tid; c < m; c += nt) {
      double w = 0.0;
      for (int r = j; r < m; ++r) w += Y[(size_t)r * m + j] * Q[(size_t)r * m + c];
      w *= bj;
      for (int r = j; r < m; ++r) Q[(size_t)r * m + c] -= w * Y[(size_t)r * m + j];
    }
    __syncthreads();
  }
}

}  // namespace

namespace {

template <typename T>
void lu_gemm(fse_ctx *ctx, T *B, int N, int r0, int m, int c0, int n, int k0, int kk) {
  if (m <= 0 || n <= 0 || kk <= 0) return;
  dim3 g((m + 63) / 64, (n + 63) / 64);
  hipLaunchKernelGGL(k_lu_gemm<T>, g, dim3(256), 0, ctx->stream, B, N, r0, m, c0, n, k0, kk);
}

template <typename T>
void lu_swap(fse_ctx *ctx, T *B, int N, int c0, int c1, int k0, int k1) {
  if (c1 <= c0 || k1 <= k0) return;
  hipLaunchKernelGGL(k_lu_swap<T>, dim3((c1 - c0 + 255) / 256), dim3(256), 0, ctx->stream, B, N, c0, c1, k0,
                     k1, ctx->piv_d);
}

template <typename T>
void lu_trsm(fse_ctx *ctx, T *B, int N, int j0, int nb, int c0, int nc) {
  if (nc <= 0 || nb <= 1) return;
  hipLaunchKernelGGL(k_lu_trsm<T>, dim3((nc + 3) / 4), dim3(256), 0, ctx->stream, B, N, j0, nb, c0, nc);
}

// Leaf width for a panel of m rows: as wide as the register-resident leaf holds
// (1024 threads x RPT rows x NB columns), else kLuLeaf with the panel in global memory.
constexpr int kRegRows8 = 5, kRegRows4 = 9;

int leaf_width(int m) {
  if (m <= 1024 * kRegRows8) return 8;
  if (m <= 1024 * kRegRows4) return 4;
  return kLuLeaf;
}

template <typename T>
void lu_leaf(fse_ctx *ctx, T *B, int N, int j0, int nb) {
  const int m = N - j0;
  if (nb <= 8 && m <= 1024 * kRegRows8)
    hipLaunchKernelGGL((k_lu_leaf_reg<T, 8, kRegRows8>), dim3(1), dim3(1024), 0, ctx->stream, B, N, j0, nb,
                       ctx->piv_d, ctx->status_d);
  else if (nb <= 4 && m <= 1024 * kRegRows4)
    hipLaunchKernelGGL((k_lu_leaf_reg<T, 4, kRegRows4>), dim3(1), dim3(1024), 0, ctx->stream, B, N, j0, nb,
                       ctx->piv_d, ctx->status_d);
  else
    hipLaunchKernelGGL(k_lu_leaf<T>, dim3(1), dim3(1024), 0, ctx->stream, B, N, j0, nb, ctx->piv_d,
                       ctx->status_d);
}

// Recursive panel B[j0:N, j0:j0+nb], nb <= kLuBlock.
template <typename T>
void lu_panel(fse_ctx *ctx, T *B, int N, int j0, int nb) {
  const int lw = leaf_width(N - j0);
  if (nb <= lw) {
    lu_leaf(ctx, B, N, j0, nb);
    return;
  }
  const int n1 = ((nb / 2 + lw - 1) / lw) * lw, n2 = nb - n1;
  lu_panel(ctx, B, N, j0, n1);
  lu_swap(ctx, B, N, j0 + n1, j0 + nb, j0, j0 + n1);
  lu_trsm(ctx, B, N, j0, n1, j0 + n1, n2);
  lu_gemm(ctx, B, N, j0 + n1, N - j0 - n1, j0 + n1, n2, j0, n1);
  lu_panel(ctx, B, N, j0 + n1, n2);
  lu_swap(ctx, B, N, j0, j0 + n1, j0 + n1, j0 + nb);
}

// ---------------------------------------------------------------- mixed-precision solve
__global__ void k_narrow(size_t n, const double *__restrict__ a, float *__restrict__ b) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

__global__ void k_widen_add(int N, const float *__restrict__ d, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) x[i] += (double)d[i];
}

// r = b - A x for the row-major N x N matrix A, one wave per row, FP64
__global__ __launch_bounds__(256) void k_resid_rows(const double *__restrict__ A, int N,
                                                    const double *__restrict__ x, const double *__restrict__ b,
                                                    double *__restrict__ r) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  const double *a = A + (size_t)row * N;
  double s = 0.0;
  for (int c = lane; c < N; c += 64) s += a[c] * x[c];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) r[row] = b[row] - s;
}

template <typename T>
fse_status lu_factor_t(fse_ctx *ctx, T *A, int N, int32_t *piv) {
  FSE_TRY(reset_status(ctx));
  int32_t *const saved = ctx->piv_d;
  ctx->piv_d = piv;  // the panel routines take the pivots from the context
  T *B = A;          // B = J^T column-major
  for (int j0 = 0; j0 < N; j0 += kLuBlock) {
    const int nb = (N - j0) < kLuBlock ? (N - j0) : kLuBlock;
    lu_panel(ctx, B, N, j0, nb);
    const int c1 = j0 + nb;
    lu_swap(ctx, B, N, c1, N, j0, c1);       // trailing columns
    lu_swap(ctx, B, N, 0, j0, j0, c1);       // earlier L columns
    lu_trsm(ctx, B, N, j0, nb, c1, N - c1);
    lu_gemm(ctx, B, N, c1, N - c1, c1, N - c1, j0, nb);
  }
  ctx->piv_d = saved;
  FSE_HIP(hipGetLastError());
  DevStatus st;
  FSE_HIP(hipMemcpyAsync(&st, ctx->status_d, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  if (st.flags & DEV_SINGULAR) {
    ctx->err = "singular Jacobian in the dense LU";
    return FSE_E_SINGULAR;
  }
  return FSE_OK;
}

template <typename T>
fse_status lu_apply_t(fse_ctx *ctx, const T *A, size_t sA, int N, const int32_t *piv, size_t sp, T *rhs,
                      size_t sx, int count) {
  if (count < 1) return FSE_OK;
  // partial sums of the solved columns: [count][chunks][64]
  const size_t nchmax = (size_t)(N + kGemvChunk - 1) / kGemvChunk, spp = nchmax * 64;
  const size_t need = sizeof(T) * spp * (size_t)count;
  if (ctx->lu_part_bytes < need) {
    if (ctx->lu_part) (void)hipFree(ctx->lu_part);
    ctx->lu_part = nullptr;
    ctx->lu_part_bytes = 0;
    if (hipMalloc(&ctx->lu_part, need) != hipSuccess) {
      ctx->err = "hipMalloc failed for the substitution partial sums";
      return FSE_E_NOMEM;
    }
    ctx->lu_part_bytes = need;
  }
  T *part = (T *)ctx->lu_part;
  // U^T v = r (forward, memory rows), then L^T w = v (backward), then x = Pi^T w; every launch
  // covers the `count` systems at once
  for (int r0 = 0; r0 < N; r0 += 64) {
    const int nb = (N - r0) < 64 ? (N - r0) : 64;
    const int nch = (r0 + kGemvChunk - 1) / kGemvChunk;
    if (nch > 0)
      hipLaunchKernelGGL(k_lu_gemv<T>, dim3((nb + 3) / 4, nch, count), dim3(256), 0, ctx->stream, A, N, r0, nb, 0,
                         r0, rhs, part, sA, sx, spp);
    hipLaunchKernelGGL(k_lu_diag<T>, dim3(count), dim3(64), 0, ctx->stream, A, N, r0, nb, false, rhs, part, nch,
                       sA, sx, spp);
  }
  const int last = ((N - 1) / 64) * 64;
  for (int r0 = last; r0 >= 0; r0 -= 64) {
    const int nb = (N - r0) < 64 ? (N - r0) : 64;
    const int nch = (N - r0 - nb + kGemvChunk - 1) / kGemvChunk;
    if (nch > 0)
      hipLaunchKernelGGL(k_lu_gemv<T>, dim3((nb + 3) / 4, nch, count), dim3(256), 0, ctx->stream, A, N, r0, nb,
                         r0 + nb, N, rhs, part, sA, sx, spp);
    hipLaunchKernelGGL(k_lu_diag<T>, dim3(count), dim3(64), 0, ctx->stream, A, N, r0, nb, true, rhs, part, nch,
                       sA, sx, spp);
  }
  const size_t lds = N <= kUnpermLds ? sizeof(T) * N : 0;
  if (lds > 64 * 1024)
    FSE_HIP(hipFuncSetAttribute((const void *)k_lu_unpermute<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(T) * kUnpermLds)));
  hipLaunchKernelGGL(k_lu_unpermute<T>, dim3(count), dim3(1024), lds, ctx->stream, rhs, N, piv, sx, sp);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status ensure_pivots(fse_ctx *ctx, int N) {
  if (ctx->piv_n < N) {
    if (ctx->piv_d) (void)hipFree(ctx->piv_d);
    ctx->piv_d = nullptr;
    ctx->piv_n = 0;
    if (hipMalloc((void **)&ctx->piv_d, sizeof(int32_t) * N) != hipSuccess) {
      ctx->err = "hipMalloc failed for the pivots";
      return FSE_E_NOMEM;
    }
    ctx->piv_n = N;
  }
  return FSE_OK;
}

}  // namespace

fse_status dense_lu_factor(fse_ctx *ctx, double *A, int N, int32_t *piv) { return lu_factor_t(ctx, A, N, piv); }

fse_status dense_lu_apply_batched(fse_ctx *ctx, const double *A, size_t sA, int N, const int32_t *piv,
                                  size_t sp, double *rhs, size_t sx, int count) {
  return lu_apply_t(ctx, A, sA, N, piv, sp, rhs, sx, count);
}

fse_status dense_lu_apply(fse_ctx *ctx, const double *A, int N, const int32_t *piv, double *rhs) {
  return dense_lu_apply_batched(ctx, A, 0, N, piv, 0, rhs, 0, 1);
}

// Mixed-precision dense solve (FP32 LU, FP64 iterative refinement): A (row-major FP64, kept)
// is rounded to FP32 and factored; then d = LU32^-1 r, x += d, r = b - A x in FP64 until
// ||r|| <= 1e-10 ||b||: an inexact Newton correction, which the outer Newton iteration on the
// FP64 shooting residual refines further.  If the refinement stalls above that (A too
// ill-conditioned for the FP32 factor) or the FP32 factor is singular, the FP64 LU solves the
// system instead.
fse_status dense_lu_solve_refined(fse_ctx *ctx, double *A, int N, double *rhs) {
  constexpr int kMaxRefine = 10;
  FSE_TRY(ensure_pivots(ctx, N));
  const size_t nn = (size_t)N * N;
  if (ctx->lu32_elems < nn + N) {
    if (ctx->lu32) (void)hipFree(ctx->lu32);
    ctx->lu32 = nullptr;
    ctx->lu32_elems = 0;
    if (hipMalloc((void **)&ctx->lu32, sizeof(float) * (nn + N)) != hipSuccess) {
      ctx->err = "hipMalloc failed for the FP32 factor";
      return FSE_E_NOMEM;
    }
    ctx->lu32_elems = nn + N;
  }
  if (ctx->ir_elems < 3 * (size_t)N) {
    if (ctx->ir) (void)hipFree(ctx->ir);
    ctx->ir = nullptr;
    ctx->ir_elems = 0;
    if (hipMalloc((void **)&ctx->ir, sizeof(double) * 3 * N) != hipSuccess) {
      ctx->err = "hipMalloc failed for the refinement vectors";
      return FSE_E_NOMEM;
    }
    ctx->ir_elems = 3 * (size_t)N;
  }
  float *A32 = ctx->lu32, *d32 = ctx->lu32 + nn;
  double *b = ctx->ir, *x = b + N, *r = x + N;
  const int nbk = (N + 255) / 256;
  hipLaunchKernelGGL(k_narrow, dim3(4096), dim3(256), 0, ctx->stream, nn, A, A32);
  FSE_HIP(hipGetLastError());
  ctx->last_refine = -1;
  const fse_status fs = lu_factor_t(ctx, A32, N, ctx->piv_d);
  if (fs != FSE_OK && fs != FSE_E_SINGULAR) return fs;
  if (fs == FSE_OK) {
    FSE_HIP(hipMemcpyAsync(b, rhs, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
    FSE_HIP(hipMemcpyAsync(r, rhs, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
    FSE_HIP(hipMemsetAsync(x, 0, sizeof(double) * N, ctx->stream));
    double nb = 0.0;
    FSE_TRY(launch_norm(ctx, b, (size_t)N, &nb));
    if (!(nb > 0.0)) {
      FSE_HIP(hipMemsetAsync(rhs, 0, sizeof(double) * N, ctx->stream));
      FSE_HIP(hipStreamSynchronize(ctx->stream));
      ctx->last_refine = 0;
      return FSE_OK;
    }
    double prev = INFINITY, nr = INFINITY;
    int it = 0;
    for (; it < kMaxRefine; ++it) {
      hipLaunchKernelGGL(k_narrow, dim3(nbk), dim3(256), 0, ctx->stream, (size_t)N, r, d32);
      FSE_TRY(lu_apply_t(ctx, (const float *)A32, 0, N, ctx->piv_d, 0, d32, 0, 1));
      hipLaunchKernelGGL(k_widen_add, dim3(nbk), dim3(256), 0, ctx->stream, N, d32, x);
      hipLaunchKernelGGL(k_resid_rows, dim3((N + 3) / 4), dim3(256), 0, ctx->stream, A, N, x, b, r);
      FSE_HIP(hipGetLastError());
      FSE_TRY(launch_norm(ctx, r, (size_t)N, &nr));
      if (nr <= 1e-10 * nb || !(nr < 0.5 * prev)) break;
      prev = nr;
    }
    if (nr <= 1e-10 * nb) {
      FSE_HIP(hipMemcpyAsync(rhs, x, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
      FSE_HIP(hipStreamSynchronize(ctx->stream));
      ctx->last_refine = it + 1;
      return FSE_OK;
    }
  }
  // the FP32 factor does not carry this system: plain FP64 LU (A is still intact)
  return dense_lu_solve(ctx, A, N, rhs);
}

fse_status newton_dense_solve(fse_ctx *ctx, double *A, int N, double *rhs) {
  return ctx->prec == FSE_PREC_MIXED_FP32 ? dense_lu_solve_refined(ctx, A, N, rhs) : dense_lu_solve(ctx, A, N, rhs);
}

fse_status dense_lu_solve(fse_ctx *ctx, double *A, int N, double *rhs) {
  if (ctx->piv_n < N) {
    if (ctx->piv_d) (void)hipFree(ctx->piv_d);
    ctx->piv_d = nullptr;
    ctx->piv_n = 0;
    if (hipMalloc((void **)&ctx->piv_d, sizeof(int32_t) * N) != hipSuccess) {
      ctx->err = "hipMalloc failed for the pivots";
      return FSE_E_NOMEM;
    }
    ctx->piv_n = N;
  }
  FSE_TRY(dense_lu_factor(ctx, A, N, ctx->piv_d));
  FSE_TRY(dense_lu_apply(ctx, A, N, ctx->piv_d, rhs));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status launch_lincomb(fse_ctx *ctx, int N, const double *x, double alpha, const double *d, double *y) {
  hipLaunchKernelGGL(k_lincomb, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, N, x, alpha, d, y);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_axpby(fse_ctx *ctx, int N, double a, const double *x, double b, const double *z, double *y) {
  hipLaunchKernelGGL(k_axpby, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, N, a, x, b, z, y);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status launch_axpy(fse_ctx *ctx, int N, double alpha, const double *x, double *y) {
  hipLaunchKernelGGL(k_axpy, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, N, alpha, x, y);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

fse_status lyapunov_qr(fse_ctx *ctx, const double *PhiQU, const double *omega_h, int N_Ly,
                       const double *Q0, double *sigma_h) {
  const int n = ctx->n, m = 2 * n, U = ctx->U, St = ctx->St, d = ctx->d, dm1 = d - 1;
  const size_t NIJ = (size_t)m * m;
  const double w1 = omega_h[0];
  // trigonometric rows H(k~, 2 pi (i-1) rho) for every Gram-Schmidt step (host, Eq. 11)
  std::vector<double> H((size_t)N_Ly * U);
  for (int i = 0; i < N_Ly; ++i) {
    H[(size_t)i * U] = 1.0;
    for (int l = 0; l < ctx->L; ++l) {
      double th = 0.0;
      for (int j = 0; j < dm1; ++j) {
        const double rho = omega_h[1 + j] / w1;
        // reduce (i-1) rho mod 1 before scaling to keep the argument small
        double fr = (double)i * rho;
        fr -= std::floor(fr);
        th += (double)ctx->ktable[(size_t)l * dm1 + j] * fr;
      }
      th *= 2.0 * M_PI;
      H[(size_t)i * U + 2 * l + 1] = std::cos(th);
      H[(size_t)i * U + 2 * l + 2] = std::sin(th);
    }
  }
  double *Ph = nullptr, *Hd = nullptr, *Psi = nullptr, *Y = nullptr, *Qm = nullptr, *beta = nullptr,
         *acc = nullptr;
  auto cleanup = [&]() {
    for (double *p : {Ph, Hd, Psi, Y, Qm, beta, acc})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc((void **)&Ph, sizeof(double) * NIJ * U) != hipSuccess ||
      hipMalloc((void **)&Hd, sizeof(double) * H.size()) != hipSuccess ||
      hipMalloc((void **)&Psi, sizeof(double) * NIJ) != hipSuccess ||
      hipMalloc((void **)&Y, sizeof(double) * NIJ) != hipSuccess ||
      hipMalloc((void **)&Qm, sizeof(double) * NIJ) != hipSuccess ||
      hipMalloc((void **)&beta, sizeof(double) * m) != hipSuccess ||
      hipMalloc((void **)&acc, sizeof(double) * m) != hipSuccess) {
    cleanup();
    ctx->err = "hipMalloc failed in the Lyapunov sweep";
    return FSE_E_NOMEM;
  }
  hipError_t e = reset_status(ctx) == FSE_OK ? hipSuccess : hipErrorUnknown;
  if (e == hipSuccess) e = hipMemcpyAsync(Hd, H.data(), sizeof(double) * H.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(acc, 0, sizeof(double) * m, ctx->stream);
  if (e == hipSuccess) {
    if (Q0) {
      e = hipMemcpyAsync(Qm, Q0, sizeof(double) * NIJ, hipMemcpyDeviceToDevice, ctx->stream);
    } else {
      std::vector<double> I(NIJ, 0.0);
      for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
      e = hipMemcpyAsync(Qm, I.data(), sizeof(double) * NIJ, hipMemcpyHostToDevice, ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
  }
  if (e != hipSuccess) {
    cleanup();
    ctx->err = std::string("HIP error ") + hipGetErrorString(e);
    return FSE_E_DEVICE;
  }
  const size_t tot = NIJ * U;
  hipLaunchKernelGGL(k_psi_hat, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, PhiQU,
                     ctx->Gi_d, n, U, St, w1, Ph);
  dim3 gg((m + 63) / 64, (m + 63) / 64);
  for (int i = 0; i < N_Ly; ++i) {
    hipLaunchKernelGGL(k_psi_interp, dim3((unsigned)((NIJ + 255) / 256)), dim3(256), 0, ctx->stream, Ph,
                       Hd + (size_t)i * U, U, NIJ, Psi);
    hipLaunchKernelGGL(k_gemm_sq, gg, dim3(256), 0, ctx->stream, Psi, Qm, m, Y);
    hipLaunchKernelGGL(k_householder, dim3(1), dim3(1024), 0, ctx->stream, Y, m, Qm, beta, acc,
                       ctx->status_d);
  }
  std::vector<double> acc_h(m);
  DevStatus st;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(acc_h.data(), acc, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&st, ctx->status_d, sizeof(st), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  cleanup();
  if (e != hipSuccess) {
    ctx->err = std::string("HIP error ") + hipGetErrorString(e);
    return FSE_E_DEVICE;
  }
  if (st.flags & DEV_SINGULAR) {
    ctx->err = "zero column in the Lyapunov QR";
    return FSE_E_SINGULAR;
  }
  const double T1 = 2.0 * M_PI / w1;
  for (int h = 0; h < m; ++h) sigma_h[h] = acc_h[h] / ((double)N_Ly * T1);
  return FSE_OK;
}
