// Dense FP64 linear algebra for the shooting Newton step (Sec. 3.3 step 6) and
// the Lyapunov exponents (App. F) on gfx950.
#include <cmath>
#include <vector>

#include "fse_internal.h"

namespace {

// ---------------------------------------------------------------- LU with partial pivoting
// Row-major A (N x N).  Panel of kb columns starting at k0 factored by one block;
// full-row swaps are applied to A and to the right-hand side immediately.
__global__ __launch_bounds__(1024) void k_lu_panel(double *__restrict__ A, int N, int k0, int kb,
                                                   double *__restrict__ rhs, DevStatus *st) {
  __shared__ double sv[16];
  __shared__ int si[16];
  __shared__ int piv_s;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  for (int j = k0; j < k0 + kb; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < N; i += nt) {
      const double v = fabs(A[(size_t)i * N + j]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o);
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
      double b = sv[0];
      int ix = si[0];
      for (int w = 1; w < (nt >> 6); ++w)
        if (sv[w] > b || (sv[w] == b && si[w] < ix)) {
          b = sv[w];
          ix = si[w];
        }
      piv_s = ix;
      if (!(b > 0.0) || !isfinite(b)) atomicOr(&st->flags, (int)DEV_SINGULAR);
    }
    __syncthreads();
    const int p = piv_s;
    if (p != j) {
      for (int c = tid; c < N; c += nt) {
        const double t = A[(size_t)j * N + c];
        A[(size_t)j * N + c] = A[(size_t)p * N + c];
        A[(size_t)p * N + c] = t;
      }
      if (tid == 0) {
        const double t = rhs[j];
        rhs[j] = rhs[p];
        rhs[p] = t;
      }
    }
    __syncthreads();
    const double inv = 1.0 / A[(size_t)j * N + j];
    for (int i = j + 1 + tid; i < N; i += nt) {
      const double l = A[(size_t)i * N + j] * inv;
      A[(size_t)i * N + j] = l;
      for (int c = j + 1; c < k0 + kb; ++c) A[(size_t)i * N + c] -= l * A[(size_t)j * N + c];
    }
    __syncthreads();
  }
}

// A12 <- L11^-1 A12 (unit lower L11 of the panel), one thread per column.
__global__ void k_lu_trsm(double *__restrict__ A, int N, int k0, int kb) {
  const int c = k0 + kb + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  for (int r = k0 + 1; r < k0 + kb; ++r) {
    double v = A[(size_t)r * N + c];
    for (int t = k0; t < r; ++t) v -= A[(size_t)r * N + t] * A[(size_t)t * N + c];
    A[(size_t)r * N + c] = v;
  }
}

// A22 -= A21 A12, 64 x 64 tiles, kb <= 64 inner.
__global__ __launch_bounds__(256) void k_lu_gemm(double *__restrict__ A, int N, int k0, int kb) {
  __shared__ double As[64][65];
  __shared__ double Bs[64][65];
  const int r0 = k0 + kb + blockIdx.y * 64;
  const int c0 = k0 + kb + blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int rr = e / 64, kk = e % 64;
    As[rr][kk] = (r0 + rr < N && kk < kb) ? A[(size_t)(r0 + rr) * N + k0 + kk] : 0.0;
    const int k2 = e / 64, cc = e % 64;
    Bs[k2][cc] = (k2 < kb && c0 + cc < N) ? A[(size_t)(k0 + k2) * N + c0 + cc] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int k = 0; k < kb; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = As[ty * 4 + i][k];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx * 4 + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty * 4 + i;
    if (r >= N) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tx * 4 + j;
      if (c < N) A[(size_t)r * N + c] -= acc[i][j];
    }
  }
}

// Triangular solves with the packed LU (unit lower L, upper U), one block.
__global__ __launch_bounds__(1024) void k_lu_substitute(const double *__restrict__ A, int N,
                                                        double *__restrict__ x) {
  __shared__ double red[16];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = tid; j < i; j += nt) s += A[(size_t)i * N + j] * x[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < (nt >> 6); ++w) t += red[w];
      x[i] -= t;
    }
    __syncthreads();
  }
  for (int i = N - 1; i >= 0; --i) {
    double s = 0.0;
    for (int j = i + 1 + tid; j < N; j += nt) s += A[(size_t)i * N + j] * x[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < (nt >> 6); ++w) t += red[w];
      x[i] = (x[i] - t) / A[(size_t)i * N + i];
    }
    __syncthreads();
  }
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

fse_status dense_lu_solve(fse_ctx *ctx, double *A, int N, double *rhs) {
  FSE_TRY(reset_status(ctx));
  const int nb = 64;
  for (int k0 = 0; k0 < N; k0 += nb) {
    const int kb = (N - k0) < nb ? (N - k0) : nb;
    hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(1024), 0, ctx->stream, A, N, k0, kb, rhs, ctx->status_d);
    const int rest = N - k0 - kb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_lu_trsm, dim3((rest + 127) / 128), dim3(128), 0, ctx->stream, A, N, k0, kb);
      dim3 g((rest + 63) / 64, (rest + 63) / 64);
      hipLaunchKernelGGL(k_lu_gemm, g, dim3(256), 0, ctx->stream, A, N, k0, kb);
    }
  }
  hipLaunchKernelGGL(k_lu_substitute, dim3(1), dim3(1024), 0, ctx->stream, A, N, rhs);
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

fse_status launch_lincomb(fse_ctx *ctx, int N, const double *x, double alpha, const double *d, double *y) {
  hipLaunchKernelGGL(k_lincomb, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, N, x, alpha, d, y);
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
