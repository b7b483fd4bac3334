// Learned predictor of initial shooting iterates: snapshot POD of converged Z(0) and a
// GELU multilayer perceptron from continuation parameters to POD coefficients, with its
// forward, backward and AdamW kernels.  FP64 for the POD, FP32 for the network.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "fse_internal.h"

struct fse_learned {
  fse_ctx *ctx = nullptr;
  int n_in = 0, H = 0, rank = 0, N = 0;
  int64_t np = 0;
  int off[6] = {0, 0, 0, 0, 0, 0};  // W1 b1 W2 b2 W3 b3 offsets in the flat parameter array
  float *par = nullptr, *grd = nullptr, *mom = nullptr, *vel = nullptr;
  int t = 0;
  // activations and gradients for up to kMaxB rows
  float *x = nullptr, *z1 = nullptr, *a1 = nullptr, *z2 = nullptr, *a2 = nullptr, *y = nullptr;
  float *tg = nullptr, *dy = nullptr, *d2 = nullptr, *d1 = nullptr, *dx = nullptr;
  double *loss_d = nullptr;
  // POD
  int m_pod = 0, r_eff = 0;
  double *mean = nullptr, *modes = nullptr, *gram = nullptr, *V = nullptr, *coef = nullptr, *cvec = nullptr;
  // normalisation of inputs and POD coefficients (training set statistics)
  std::vector<double> mu_p, sd_p, mu_c, sd_c;
  bool trained = false;
};

namespace {

constexpr int kMaxB = 256;
constexpr int kMaxSnap = 128;

// C[m][n] (+)= sum_k A(m, k) B(k, n) (+ bias[n]); strided operands, 16 x 16 tiles in LDS.
__global__ __launch_bounds__(256) void k_gemm_f32(int M, int Nn, int K, const float *__restrict__ A, int am,
                                                  int ak, const float *__restrict__ B, int bk, int bn,
                                                  float *__restrict__ C, int ldc, const float *__restrict__ bias,
                                                  int accumulate) {
  __shared__ float As[16][17];
  __shared__ float Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
  float acc = 0.0f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (m < M && ka < K) ? A[(size_t)m * am + (size_t)ka * ak] : 0.0f;
    Bs[ty][tx] = (kb < K && n < Nn) ? B[(size_t)kb * bk + (size_t)n * bn] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bs[k][tx];
    __syncthreads();
  }
  if (m < M && n < Nn) {
    float v = acc + (bias ? bias[n] : 0.0f);
    if (accumulate) v += C[(size_t)m * ldc + n];
    C[(size_t)m * ldc + n] = v;
  }
}

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_df(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void k_gelu(int n, const float *__restrict__ z, float *__restrict__ a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = gelu_f(z[i]);
}

// g <- g * gelu'(z)
__global__ void k_gelu_back(int n, const float *__restrict__ z, float *__restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] *= gelu_df(z[i]);
}

// dy = 2 (y - t) / count; loss = mean (y - t)^2 (one block)
__global__ __launch_bounds__(1024) void k_mse(int count, const float *__restrict__ y, const float *__restrict__ t,
                                              float *__restrict__ dy, double *__restrict__ loss) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const float r = y[i] - t[i];
    dy[i] = 2.0f * r / (float)count;
    s += (double)r * (double)r;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
    *loss = tot / (double)count;
  }
}

// out[n] = sum_m g[m][n] (bias gradients)
__global__ void k_colsum(int M, int Nn, const float *__restrict__ g, float *__restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Nn) return;
  float s = 0.0f;
  for (int m = 0; m < M; ++m) s += g[(size_t)m * Nn + n];
  out[n] = s;
}

// decoupled-weight-decay Adam over the flat parameter array
__global__ void k_adamw(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1,
                        float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

// ------------------------------------------------------------------ POD (FP64)
__global__ void k_snap_mean(int m, int N, const double *__restrict__ X, double *__restrict__ mean) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int a = 0; a < m; ++a) s += X[(size_t)a * N + i];
  mean[i] = s / (double)m;
}

// G[a][b] = <x_a - mean, x_b - mean>, one wave per pair a <= b
__global__ __launch_bounds__(256) void k_gram(int m, int N, const double *__restrict__ X,
                                              const double *__restrict__ mean, double *__restrict__ G) {
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (pair >= m * m) return;
  const int a = pair / m, b = pair % m;
  if (b < a) return;
  const double *xa = X + (size_t)a * N, *xb = X + (size_t)b * N;
  double s = 0.0;
  for (int i = lane; i < N; i += 64) s += (xa[i] - mean[i]) * (xb[i] - mean[i]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) {
    G[(size_t)a * m + b] = s;
    G[(size_t)b * m + a] = s;
  }
}

// Cyclic Jacobi eigen-solver of the symmetric m x m matrix G (m <= kMaxSnap), one block:
// G kept in LDS, eigenvectors accumulated in V (global, row j = component j).  On return
// the diagonal of G (copied to lam) holds the eigenvalues.
__global__ __launch_bounds__(1024) void k_jacobi(int m, double *__restrict__ G, double *__restrict__ V,
                                                 double *__restrict__ lam, int max_sweeps) {
  extern __shared__ double A[];  // [m][m+1]
  __shared__ double sc, ss, st;
  __shared__ int s_done;
  const int ld = m + 1, tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < m * m; e += nt) {
    A[(e / m) * ld + (e % m)] = G[e];
    V[e] = ((e / m) == (e % m)) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) {
      double off = 0.0, dia = 0.0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          const double v = A[i * ld + j] * A[i * ld + j];
          if (i == j)
            dia += v;
          else
            off += v;
        }
      s_done = (off <= 1e-30 * dia) ? 1 : 0;
    }
    __syncthreads();
    if (s_done) break;
    for (int p = 0; p < m - 1; ++p) {
      for (int q = p + 1; q < m; ++q) {
        if (tid == 0) {
          const double apq = A[p * ld + q];
          double c = 1.0, s = 0.0, t = 0.0;
          if (fabs(apq) > 1e-300) {
            const double tau = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
          sc = c;
          ss = s;
          st = t;
        }
        __syncthreads();
        const double c = sc, s = ss, t = st;
        __syncthreads();  // every thread holds (c, s, t) before thread 0 may overwrite them
        if (s != 0.0) {
          // columns p, q of A and V
          for (int k = tid; k < m; k += nt) {
            if (k != p && k != q) {
              const double akp = A[k * ld + p], akq = A[k * ld + q];
              A[k * ld + p] = c * akp - s * akq;
              A[k * ld + q] = s * akp + c * akq;
            }
            const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
            V[(size_t)k * m + p] = c * vkp - s * vkq;
            V[(size_t)k * m + q] = s * vkp + c * vkq;
          }
          __syncthreads();
          // rows p, q mirror the columns; the 2 x 2 block gets the rotated diagonal
          for (int k = tid; k < m; k += nt) {
            if (k != p && k != q) {
              A[p * ld + k] = A[k * ld + p];
              A[q * ld + k] = A[k * ld + q];
            }
          }
          if (tid == 0) {
            const double apq = A[p * ld + q];
            A[p * ld + p] -= t * apq;
            A[q * ld + q] += t * apq;
            A[p * ld + q] = 0.0;
            A[q * ld + p] = 0.0;
          }
          __syncthreads();
        }
      }
    }
  }
  for (int i = tid; i < m; i += nt) lam[i] = A[i * ld + i];
}

// modes[i][r] = sum_j (X[j][i] - mean[i]) V[j][ord[r]] / sigma_r for r < r_eff, else 0
__global__ void k_pod_modes(int m, int N, int rank, int r_eff, const double *__restrict__ X,
                            const double *__restrict__ mean, const double *__restrict__ V,
                            const int *__restrict__ ord, const double *__restrict__ sig,
                            double *__restrict__ modes) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)N * rank) return;
  const int r = idx % rank;
  const int i = idx / rank;
  double s = 0.0;
  if (r < r_eff) {
    const int c = ord[r];
    for (int j = 0; j < m; ++j) s += (X[(size_t)j * N + i] - mean[i]) * V[(size_t)j * m + c];
    s /= sig[r];
  }
  modes[idx] = s;
}

// coef[j][r] = <modes[:, r], x_j - mean>, one wave per (j, r)
__global__ __launch_bounds__(256) void k_pod_coef(int m, int N, int rank, const double *__restrict__ X,
                                                  const double *__restrict__ mean,
                                                  const double *__restrict__ modes, double *__restrict__ coef) {
  const int pr = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (pr >= m * rank) return;
  const int j = pr / rank, r = pr % rank;
  double s = 0.0;
  for (int i = lane; i < N; i += 64) s += modes[(size_t)i * rank + r] * (X[(size_t)j * N + i] - mean[i]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) coef[pr] = s;
}

// ------------------------------------------------------------------ BF16 MFMA inference
// Dense layer Y[m][n] = act(sum_k X[m][k] W[n][k] + b[n]) with X and W rounded to bfloat16
// (nearest, ties to even) as they are loaded and the products accumulated in FP32 by
// v_mfma_f32_16x16x16_bf16.  One wave per 16 x 16 output tile, four waves along n.  Operand
// layout of that instruction: lane l supplies A[l % 16][4 (l / 16) + i] and
// B[4 (l / 16) + i][l % 16], i < 4, and receives C[4 (l / 16) + i][l % 16].
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline short f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__global__ __launch_bounds__(256) void k_dense_bf16(int M, int N, int K, const float *__restrict__ X,
                                                    const float *__restrict__ W, const float *__restrict__ bias,
                                                    int gelu, float *__restrict__ Y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 16, n0 = (blockIdx.x * 4 + wave) * 16;
  if (n0 >= N) return;  // the whole wave leaves together
  const int r = lane & 15, kg = (lane >> 4) * 4;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + kg + i;
      a[i] = (m0 + r < M && k < K) ? f32_to_bf16(X[(size_t)(m0 + r) * K + k]) : (short)0;
      b[i] = (n0 + r < N && k < K) ? f32_to_bf16(W[(size_t)(n0 + r) * K + k]) : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + kg + i, n = n0 + r;
    if (m < M && n < N) {
      float v = acc[i] + bias[n];
      Y[(size_t)m * N + n] = gelu ? gelu_f(v) : v;
    }
  }
}

// Z[p][i] = mean[i] + sum_r modes[i][r] c[p][r]
__global__ void k_pod_expand_batch(int P, int N, int rank, const double *__restrict__ mean,
                                   const double *__restrict__ modes, const double *__restrict__ c,
                                   double *__restrict__ Z) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)P * N) return;
  const int p = (int)(idx / N), i = (int)(idx % N);
  double s = mean[i];
  for (int r = 0; r < rank; ++r) s += modes[(size_t)i * rank + r] * c[(size_t)p * rank + r];
  Z[idx] = s;
}

// Z[i] = mean[i] + sum_r modes[i][r] c[r]
__global__ void k_pod_expand(int N, int rank, const double *__restrict__ mean, const double *__restrict__ modes,
                             const double *__restrict__ c, double *__restrict__ Z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = mean[i];
  for (int r = 0; r < rank; ++r) s += modes[(size_t)i * rank + r] * c[r];
  Z[i] = s;
}

// ------------------------------------------------------------------ host helpers
void gemm(fse_learned *m, int M, int Nn, int K, const float *A, int am, int ak, const float *B, int bk, int bn,
          float *C, int ldc, const float *bias, bool acc) {
  dim3 g((Nn + 15) / 16, (M + 15) / 16);
  hipLaunchKernelGGL(k_gemm_f32, g, dim3(256), 0, m->ctx->stream, M, Nn, K, A, am, ak, B, bk, bn, C, ldc, bias,
                     acc ? 1 : 0);
}

template <typename T>
fse_status dalloc(fse_ctx *ctx, T **p, size_t count) {
  if (hipMalloc((void **)p, sizeof(T) * (count ? count : 1)) != hipSuccess) {
    ctx->err = "hipMalloc failed in the learned predictor";
    return FSE_E_NOMEM;
  }
  return FSE_OK;
}

// forward pass for B rows of m->x: z1, a1, z2, a2, y
void forward(fse_learned *m, int B) {
  const int H = m->H, nin = m->n_in, R = m->rank;
  const float *W1 = m->par + m->off[0], *b1 = m->par + m->off[1];
  const float *W2 = m->par + m->off[2], *b2 = m->par + m->off[3];
  const float *W3 = m->par + m->off[4], *b3 = m->par + m->off[5];
  hipStream_t s = m->ctx->stream;
  gemm(m, B, H, nin, m->x, nin, 1, W1, 1, nin, m->z1, H, b1, false);
  hipLaunchKernelGGL(k_gelu, dim3((B * H + 255) / 256), dim3(256), 0, s, B * H, m->z1, m->a1);
  gemm(m, B, H, H, m->a1, H, 1, W2, 1, H, m->z2, H, b2, false);
  hipLaunchKernelGGL(k_gelu, dim3((B * H + 255) / 256), dim3(256), 0, s, B * H, m->z2, m->a2);
  gemm(m, B, R, H, m->a2, H, 1, W3, 1, H, m->y, R, b3, false);
}

// forward pass for B rows of m->x with BF16 MFMA layers: a1, a2, y
void forward_bf16(fse_learned *m, int B) {
  const int H = m->H, nin = m->n_in, R = m->rank;
  const float *W1 = m->par + m->off[0], *b1 = m->par + m->off[1];
  const float *W2 = m->par + m->off[2], *b2 = m->par + m->off[3];
  const float *W3 = m->par + m->off[4], *b3 = m->par + m->off[5];
  hipStream_t s = m->ctx->stream;
  const dim3 blk(256);
  hipLaunchKernelGGL(k_dense_bf16, dim3((H + 63) / 64, (B + 15) / 16), blk, 0, s, B, H, nin, m->x, W1, b1, 1, m->a1);
  hipLaunchKernelGGL(k_dense_bf16, dim3((H + 63) / 64, (B + 15) / 16), blk, 0, s, B, H, H, m->a1, W2, b2, 1, m->a2);
  hipLaunchKernelGGL(k_dense_bf16, dim3((R + 63) / 64, (B + 15) / 16), blk, 0, s, B, R, H, m->a2, W3, b3, 0, m->y);
}

// loss and gradients for B rows (targets in m->tg) into m->grd
void backward(fse_learned *m, int B) {
  const int H = m->H, nin = m->n_in, R = m->rank;
  const float *W2 = m->par + m->off[2], *W3 = m->par + m->off[4];
  float *gW1 = m->grd + m->off[0], *gb1 = m->grd + m->off[1];
  float *gW2 = m->grd + m->off[2], *gb2 = m->grd + m->off[3];
  float *gW3 = m->grd + m->off[4], *gb3 = m->grd + m->off[5];
  hipStream_t s = m->ctx->stream;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, B * R, m->y, m->tg, m->dy, m->loss_d);
  // layer 3: gW3[o][i] = sum_b dy[b][o] a2[b][i]; gb3; d2 = dy W3
  gemm(m, R, H, B, m->dy, 1, R, m->a2, H, 1, gW3, H, nullptr, false);
  hipLaunchKernelGGL(k_colsum, dim3((R + 255) / 256), dim3(256), 0, s, B, R, m->dy, gb3);
  gemm(m, B, H, R, m->dy, R, 1, W3, H, 1, m->d2, H, nullptr, false);
  hipLaunchKernelGGL(k_gelu_back, dim3((B * H + 255) / 256), dim3(256), 0, s, B * H, m->z2, m->d2);
  // layer 2
  gemm(m, H, H, B, m->d2, 1, H, m->a1, H, 1, gW2, H, nullptr, false);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, B, H, m->d2, gb2);
  gemm(m, B, H, H, m->d2, H, 1, W2, H, 1, m->d1, H, nullptr, false);
  hipLaunchKernelGGL(k_gelu_back, dim3((B * H + 255) / 256), dim3(256), 0, s, B * H, m->z1, m->d1);
  // layer 1
  gemm(m, H, nin, B, m->d1, 1, H, m->x, nin, 1, gW1, nin, nullptr, false);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, B, H, m->d1, gb1);
}

void adamw(fse_learned *m, double lr, double wd) {
  m->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, m->t)), c2 = (float)(1.0 - std::pow(0.999, m->t));
  hipLaunchKernelGGL(k_adamw, dim3((unsigned)((m->np + 255) / 256)), dim3(256), 0, m->ctx->stream, m->np, m->par,
                     m->grd, m->mom, m->vel, (float)lr, b1, b2, 1e-8f, (float)wd, c1, c2);
}

}  // namespace

extern "C" {

fse_status fse_learned_create(fse_ctx *ctx, int32_t n_in, int32_t hidden, int32_t rank, fse_learned **out) {
  if (!ctx || !out || n_in < 1 || hidden < 1 || rank < 1 || n_in > 64 || hidden > 4096 || rank > 1024)
    return FSE_E_INVAL;
  *out = nullptr;
  fse_learned *m = new fse_learned();
  m->ctx = ctx;
  m->n_in = n_in;
  m->H = hidden;
  m->rank = rank;
  m->N = 2 * ctx->n * ctx->U;
  const int64_t sz[6] = {(int64_t)hidden * n_in, hidden, (int64_t)hidden * hidden, hidden,
                         (int64_t)rank * hidden, rank};
  int64_t o = 0;
  for (int i = 0; i < 6; ++i) {
    m->off[i] = (int)o;
    o += sz[i];
  }
  m->np = o;
  fse_status st = FSE_OK;
  auto A = [&](fse_status s) {
    if (st == FSE_OK) st = s;
  };
  A(dalloc(ctx, &m->par, m->np));
  A(dalloc(ctx, &m->grd, m->np));
  A(dalloc(ctx, &m->mom, m->np));
  A(dalloc(ctx, &m->vel, m->np));
  A(dalloc(ctx, &m->x, (size_t)kMaxB * n_in));
  A(dalloc(ctx, &m->z1, (size_t)kMaxB * hidden));
  A(dalloc(ctx, &m->a1, (size_t)kMaxB * hidden));
  A(dalloc(ctx, &m->z2, (size_t)kMaxB * hidden));
  A(dalloc(ctx, &m->a2, (size_t)kMaxB * hidden));
  A(dalloc(ctx, &m->y, (size_t)kMaxB * rank));
  A(dalloc(ctx, &m->tg, (size_t)kMaxB * rank));
  A(dalloc(ctx, &m->dy, (size_t)kMaxB * rank));
  A(dalloc(ctx, &m->d2, (size_t)kMaxB * hidden));
  A(dalloc(ctx, &m->d1, (size_t)kMaxB * hidden));
  A(dalloc(ctx, &m->loss_d, 1));
  A(dalloc(ctx, &m->mean, m->N));
  A(dalloc(ctx, &m->modes, (size_t)m->N * rank));
  A(dalloc(ctx, &m->gram, (size_t)kMaxSnap * kMaxSnap));
  A(dalloc(ctx, &m->V, (size_t)kMaxSnap * kMaxSnap));
  A(dalloc(ctx, &m->coef, (size_t)kMaxSnap * rank + kMaxSnap));
  A(dalloc(ctx, &m->cvec, rank));
  if (st == FSE_OK) {
    if (hipMemsetAsync(m->par, 0, sizeof(float) * m->np, ctx->stream) != hipSuccess ||
        hipMemsetAsync(m->mom, 0, sizeof(float) * m->np, ctx->stream) != hipSuccess ||
        hipMemsetAsync(m->vel, 0, sizeof(float) * m->np, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      st = FSE_E_DEVICE;
  }
  if (st != FSE_OK) {
    fse_learned_destroy(m);
    return st;
  }
  *out = m;
  return FSE_OK;
}

int64_t fse_learned_num_params(const fse_learned *m) { return m ? m->np : -1; }

int32_t fse_learned_inputs(const fse_learned *m) { return m ? m->n_in : -1; }

fse_status fse_learned_set_params(fse_learned *m, const float *params) {
  if (!m || !params) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  FSE_HIP(hipMemcpyAsync(m->par, params, sizeof(float) * m->np, hipMemcpyHostToDevice, ctx->stream));
  FSE_HIP(hipMemsetAsync(m->mom, 0, sizeof(float) * m->np, ctx->stream));
  FSE_HIP(hipMemsetAsync(m->vel, 0, sizeof(float) * m->np, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  m->t = 0;
  return FSE_OK;
}

fse_status fse_learned_get_params(const fse_learned *m, float *params) {
  if (!m || !params) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  FSE_HIP(hipMemcpyAsync(params, m->par, sizeof(float) * m->np, hipMemcpyDeviceToHost, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_learned_fit_pod(fse_learned *m, int32_t m_snap, const double *X, double *sigma) {
  if (!m || !X || m_snap < 2 || m_snap > kMaxSnap) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  const int N = m->N, ms = m_snap;
  hipStream_t s = ctx->stream;
  hipLaunchKernelGGL(k_snap_mean, dim3((N + 255) / 256), dim3(256), 0, s, ms, N, X, m->mean);
  hipLaunchKernelGGL(k_gram, dim3((ms * ms + 3) / 4), dim3(256), 0, s, ms, N, X, m->mean, m->gram);
  const size_t lds = sizeof(double) * ms * (ms + 1);
  FSE_HIP(hipFuncSetAttribute((const void *)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  double *lam_d = m->coef;  // scratch
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), lds, s, ms, m->gram, m->V, lam_d, 60);
  FSE_HIP(hipGetLastError());
  std::vector<double> lam(ms);
  FSE_HIP(hipMemcpyAsync(lam.data(), lam_d, sizeof(double) * ms, hipMemcpyDeviceToHost, s));
  FSE_HIP(hipStreamSynchronize(s));
  std::vector<int> ord(ms);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return lam[a] > lam[b]; });
  const double lmax = std::max(lam[ord[0]], 0.0);
  int r_eff = 0;
  std::vector<double> sig(m->rank, 0.0);
  for (int r = 0; r < std::min(m->rank, ms); ++r) {
    const double l = std::max(lam[ord[r]], 0.0);
    if (lmax > 0.0 && l > lmax * 1e-28) {
      sig[r] = std::sqrt(l);
      r_eff = r + 1;
    }
  }
  if (sigma)
    for (int r = 0; r < std::min(m->rank, ms); ++r) sigma[r] = std::sqrt(std::max(lam[ord[r]], 0.0));
  int *ord_d = nullptr;
  double *sig_d = nullptr;
  FSE_TRY(dalloc(ctx, &ord_d, ms));
  if (dalloc(ctx, &sig_d, m->rank) != FSE_OK) {
    (void)hipFree(ord_d);
    return FSE_E_NOMEM;
  }
  hipError_t e = hipMemcpyAsync(ord_d, ord.data(), sizeof(int) * ms, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(sig_d, sig.data(), sizeof(double) * m->rank, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    const size_t tot = (size_t)N * m->rank;
    hipLaunchKernelGGL(k_pod_modes, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ms, N, m->rank, r_eff, X,
                       m->mean, m->V, ord_d, sig_d, m->modes);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(ord_d);
  (void)hipFree(sig_d);
  if (e != hipSuccess) {
    ctx->err = std::string("HIP error ") + hipGetErrorString(e);
    return FSE_E_DEVICE;
  }
  m->m_pod = ms;
  m->r_eff = r_eff;
  m->trained = false;
  return FSE_OK;
}

fse_status fse_learned_get_pod(const fse_learned *m, double *mean, double *modes) {
  if (!m || m->m_pod == 0) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  if (mean) FSE_HIP(hipMemcpyAsync(mean, m->mean, sizeof(double) * m->N, hipMemcpyDeviceToDevice, ctx->stream));
  if (modes)
    FSE_HIP(hipMemcpyAsync(modes, m->modes, sizeof(double) * m->N * m->rank, hipMemcpyDeviceToDevice, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_learned_loss_grad(fse_learned *m, int32_t B, const float *x, const float *t, float *loss,
                                 float *grads) {
  if (!m || !x || !t || B < 1 || B > kMaxB) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  hipStream_t s = ctx->stream;
  FSE_HIP(hipMemcpyAsync(m->x, x, sizeof(float) * B * m->n_in, hipMemcpyHostToDevice, s));
  FSE_HIP(hipMemcpyAsync(m->tg, t, sizeof(float) * B * m->rank, hipMemcpyHostToDevice, s));
  forward(m, B);
  backward(m, B);
  FSE_HIP(hipGetLastError());
  double l = 0.0;
  FSE_HIP(hipMemcpyAsync(&l, m->loss_d, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grads) FSE_HIP(hipMemcpyAsync(grads, m->grd, sizeof(float) * m->np, hipMemcpyDeviceToHost, s));
  FSE_HIP(hipStreamSynchronize(s));
  if (loss) *loss = (float)l;
  return FSE_OK;
}

fse_status fse_learned_fit(fse_learned *m, int32_t B, const float *x, const float *t, int32_t steps, double lr,
                           double wd, double *loss_hist) {
  if (!m || !x || !t || B < 1 || B > kMaxB || steps < 0) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  hipStream_t s = ctx->stream;
  FSE_HIP(hipMemcpyAsync(m->x, x, sizeof(float) * B * m->n_in, hipMemcpyHostToDevice, s));
  FSE_HIP(hipMemcpyAsync(m->tg, t, sizeof(float) * B * m->rank, hipMemcpyHostToDevice, s));
  for (int ep = 0; ep < steps; ++ep) {
    forward(m, B);
    backward(m, B);
    adamw(m, lr, wd);
    if (loss_hist) FSE_HIP(hipMemcpyAsync(&loss_hist[ep], m->loss_d, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  FSE_HIP(hipGetLastError());
  FSE_HIP(hipStreamSynchronize(s));
  return FSE_OK;
}

fse_status fse_learned_train(fse_learned *m, int32_t m_snap, const double *P, const double *X, int32_t epochs,
                             double lr, double wd, double *loss_hist) {
  if (!m || !P || !X || m_snap < 2 || m_snap > kMaxSnap || epochs < 0) return FSE_E_INVAL;
  if (m->m_pod == 0) {
    m->ctx->err = "fit the POD basis before training";
    return FSE_E_INVAL;
  }
  fse_ctx *ctx = m->ctx;
  hipStream_t s = ctx->stream;
  const int R = m->rank, nin = m->n_in, ms = m_snap, N = m->N;
  // POD coefficients of the training snapshots
  hipLaunchKernelGGL(k_pod_coef, dim3((ms * R + 3) / 4), dim3(256), 0, s, ms, N, R, X, m->mean, m->modes,
                     m->coef);
  FSE_HIP(hipGetLastError());
  std::vector<double> c((size_t)ms * R);
  FSE_HIP(hipMemcpyAsync(c.data(), m->coef, sizeof(double) * c.size(), hipMemcpyDeviceToHost, s));
  FSE_HIP(hipStreamSynchronize(s));
  // Inputs: unit deviation per component (components without spread keep deviation 1).
  // Coefficients: centred and divided by one common scale, the RMS deviation of the training
  // snapshots from their mean (sqrt of the summed coefficient variances).  The modes are
  // orthonormal, so the training loss is then the mean squared error of the predicted Z(0) in the
  // POD subspace; a scale per coefficient would weight a mode that carries 1e-6 of the variance
  // like the leading one.
  m->mu_p.assign(nin, 0.0);
  m->sd_p.assign(nin, 0.0);
  m->mu_c.assign(R, 0.0);
  m->sd_c.assign(R, 0.0);
  for (int j = 0; j < ms; ++j)
    for (int k = 0; k < nin; ++k) m->mu_p[k] += P[(size_t)j * nin + k] / ms;
  for (int j = 0; j < ms; ++j)
    for (int k = 0; k < nin; ++k) {
      const double dv = P[(size_t)j * nin + k] - m->mu_p[k];
      m->sd_p[k] += dv * dv / ms;
    }
  for (int j = 0; j < ms; ++j)
    for (int r = 0; r < R; ++r) m->mu_c[r] += c[(size_t)j * R + r] / ms;
  for (int j = 0; j < ms; ++j)
    for (int r = 0; r < R; ++r) {
      const double dv = c[(size_t)j * R + r] - m->mu_c[r];
      m->sd_c[r] += dv * dv / ms;
    }
  for (double &x : m->sd_p) x = (x > 0.0) ? std::sqrt(x) : 1.0;
  double var_c = 0.0;
  for (double x : m->sd_c) var_c += x;
  const double sc = var_c > 0.0 ? std::sqrt(var_c) : 1.0;
  for (double &x : m->sd_c) x = sc;
  std::vector<float> xf((size_t)ms * nin), tf((size_t)ms * R);
  for (int j = 0; j < ms; ++j) {
    for (int k = 0; k < nin; ++k)
      xf[(size_t)j * nin + k] = (float)((P[(size_t)j * nin + k] - m->mu_p[k]) / m->sd_p[k]);
    for (int r = 0; r < R; ++r) tf[(size_t)j * R + r] = (float)((c[(size_t)j * R + r] - m->mu_c[r]) / m->sd_c[r]);
  }
  FSE_TRY(fse_learned_fit(m, ms, xf.data(), tf.data(), epochs, lr, wd, loss_hist));
  m->trained = true;
  return FSE_OK;
}

fse_status fse_learned_predict(fse_learned *m, const double *p, double *Z) {
  if (!m || !p || !Z) return FSE_E_INVAL;
  if (!m->trained) {
    m->ctx->err = "the learned predictor is not trained";
    return FSE_E_INVAL;
  }
  fse_ctx *ctx = m->ctx;
  hipStream_t s = ctx->stream;
  const int nin = m->n_in, R = m->rank;
  std::vector<float> xf(nin), yf(R);
  for (int k = 0; k < nin; ++k) xf[k] = (float)((p[k] - m->mu_p[k]) / m->sd_p[k]);
  FSE_HIP(hipMemcpyAsync(m->x, xf.data(), sizeof(float) * nin, hipMemcpyHostToDevice, s));
  forward(m, 1);
  FSE_HIP(hipMemcpyAsync(yf.data(), m->y, sizeof(float) * R, hipMemcpyDeviceToHost, s));
  FSE_HIP(hipStreamSynchronize(s));
  std::vector<double> cv(R);
  for (int r = 0; r < R; ++r) cv[r] = m->mu_c[r] + m->sd_c[r] * (double)yf[r];
  FSE_HIP(hipMemcpyAsync(m->cvec, cv.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_pod_expand, dim3((m->N + 255) / 256), dim3(256), 0, s, m->N, R, m->mean, m->modes, m->cvec,
                     Z);
  FSE_HIP(hipGetLastError());
  FSE_HIP(hipStreamSynchronize(s));
  return FSE_OK;
}

fse_status fse_learned_forward(fse_learned *m, int32_t B, const float *x, int32_t bf16, float *y) {
  if (!m || !x || !y || B < 1 || B > kMaxB) return FSE_E_INVAL;
  fse_ctx *ctx = m->ctx;
  hipStream_t s = ctx->stream;
  FSE_HIP(hipMemcpyAsync(m->x, x, sizeof(float) * B * m->n_in, hipMemcpyHostToDevice, s));
  if (bf16)
    forward_bf16(m, B);
  else
    forward(m, B);
  FSE_HIP(hipGetLastError());
  FSE_HIP(hipMemcpyAsync(y, m->y, sizeof(float) * B * m->rank, hipMemcpyDeviceToHost, s));
  FSE_HIP(hipStreamSynchronize(s));
  return FSE_OK;
}

fse_status fse_learned_predict_batch(fse_learned *m, int32_t P, const double *params, int32_t bf16, double *Z) {
  if (!m || !params || !Z || P < 1 || P > kMaxB) return FSE_E_INVAL;
  if (!m->trained) {
    m->ctx->err = "the learned predictor is not trained";
    return FSE_E_INVAL;
  }
  fse_ctx *ctx = m->ctx;
  hipStream_t s = ctx->stream;
  const int nin = m->n_in, R = m->rank;
  std::vector<float> xf((size_t)P * nin), yf((size_t)P * R);
  for (int p = 0; p < P; ++p)
    for (int k = 0; k < nin; ++k)
      xf[(size_t)p * nin + k] = (float)((params[(size_t)p * nin + k] - m->mu_p[k]) / m->sd_p[k]);
  FSE_HIP(hipMemcpyAsync(m->x, xf.data(), sizeof(float) * xf.size(), hipMemcpyHostToDevice, s));
  if (bf16)
    forward_bf16(m, P);
  else
    forward(m, P);
  FSE_HIP(hipGetLastError());
  FSE_HIP(hipMemcpyAsync(yf.data(), m->y, sizeof(float) * yf.size(), hipMemcpyDeviceToHost, s));
  FSE_HIP(hipStreamSynchronize(s));
  std::vector<double> cv((size_t)P * R);
  for (int p = 0; p < P; ++p)
    for (int r = 0; r < R; ++r) cv[(size_t)p * R + r] = m->mu_c[r] + m->sd_c[r] * (double)yf[(size_t)p * R + r];
  double *cd = nullptr;
  if (hipMalloc((void **)&cd, sizeof(double) * cv.size()) != hipSuccess) {
    ctx->err = "hipMalloc failed for the batch coefficients";
    return FSE_E_NOMEM;
  }
  hipError_t e = hipMemcpyAsync(cd, cv.data(), sizeof(double) * cv.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    const size_t tot = (size_t)P * m->N;
    hipLaunchKernelGGL(k_pod_expand_batch, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, P, m->N, R, m->mean,
                       m->modes, cd, Z);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(cd);
  FSE_HIP(e);
  return FSE_OK;
}

void fse_learned_destroy(fse_learned *m) {
  if (!m) return;
  void *ptrs[] = {m->par, m->grd, m->mom, m->vel, m->x,    m->z1,    m->a1,   m->z2,   m->a2,
                  m->y,   m->tg,  m->dy,  m->d2,  m->d1,   m->loss_d, m->mean, m->modes, m->gram,
                  m->V,   m->coef, m->cvec};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

}  // extern "C"
