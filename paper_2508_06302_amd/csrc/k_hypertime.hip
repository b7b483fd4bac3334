// FSE-Shooting in the hyper-time domain (Sec. 3.4, Eq. FSES_T) on gfx950.
//
// The unknowns are the sampled initial states zbar(0) [2n][S~] themselves; the residual is
//     R = (I (x) A) zbar(2 pi) - zbar(0),   A = Gamma R(rho) Gamma^-1  (S~ x S~),
// with zbar(2 pi) from the same trajectory kernels as the multi-frequency form, and its
// Jacobian J[(i, s), (j, t)] = A[s, t] Phi_t[i, j] - delta (unknowns state-major,
// (i, s) -> i S~ + s).  A is built on the device per point from Gamma, Gamma^-1 and the
// rotation angles of Eq. (14).  With unknown frequencies the Newton step is bordered (k_ht_border).
#include <algorithm>
#include <cmath>
#include <vector>

#include "fse_internal.h"

namespace {

// qhist[0] / u0 from samples zbar(0) [B][2n][S~]: trajectory w = b S~ + s
__global__ void k_samples_in(const double *__restrict__ z0, int n, int St, int W, int ldw,
                             double *__restrict__ q0, double *__restrict__ u0) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;  // state row 0..2n-1
  if (w >= W) return;
  const int b = w / St, s = w - (w / St) * St;
  const double v = z0[((size_t)b * 2 * n + i) * St + s];
  if (i < n)
    q0[(size_t)i * ldw + w] = v;
  else
    u0[(size_t)(i - n) * ldw + w] = v;
}

// RGi[b][l][t] = (R(rho_b) Gamma^-1)[l][t]: row 0 as is, each pair (a, a + 1) rotated
__global__ void k_ht_rgi(const double *__restrict__ Gi, const double *__restrict__ rot, int U, int St, int Lm,
                         double *__restrict__ RGi) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= U * St) return;
  const int l = idx / St, t = idx - (idx / St) * St;
  double v;
  if (l == 0) {
    v = Gi[t];
  } else {
    const int p = (l - 1) / 2, a = 2 * p + 1;
    const double al = rot[(size_t)b * Lm + p], c = cos(al), sn = sin(al);
    const double ga = Gi[(size_t)a * St + t], gb = Gi[(size_t)(a + 1) * St + t];
    v = (l == a) ? c * ga - sn * gb : sn * ga + c * gb;
  }
  RGi[(size_t)b * U * St + idx] = v;
}

// A[b][s][t] = sum_l Gamma[s][l] RGi[b][l][t]
__global__ void k_ht_A(const double *__restrict__ G, const double *__restrict__ RGi, int U, int St,
                       double *__restrict__ A) {
  const int b = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= St * St) return;
  const int s = idx / St, t = idx - (idx / St) * St;
  const double *g = G + (size_t)s * U;
  const double *r = RGi + (size_t)b * U * St + t;
  double acc = 0.0;
  for (int l = 0; l < U; ++l) acc += g[l] * r[(size_t)l * St];
  A[(size_t)b * St * St + idx] = acc;
}

// R[b][i][s] = sum_t A[b][s][t] zT[i][b S~ + t] - z0[b][i][s]
__global__ void k_ht_residual(const double *__restrict__ zT, int ldw, const double *__restrict__ A,
                              const double *__restrict__ z0, int n2, int St, int B, double *__restrict__ R) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)n2 * St;
  if (idx >= per * B) return;
  const int b = (int)(idx / per);
  const size_t r = idx - (size_t)b * per;
  const int i = (int)(r / St), s = (int)(r % St);
  const double *a = A + ((size_t)b * St + s) * St;
  const double *z = zT + (size_t)i * ldw + (size_t)b * St;
  double acc = 0.0;
  for (int t = 0; t < St; ++t) acc += a[t] * z[t];
  R[idx] = acc - z0[idx];
}

// J[(i, s), (j, t)] = A[s][t] Phi_{b S~ + t}[i][j] - delta for one point b (grid-stride)
__global__ void k_ht_jac(const double *__restrict__ A, const double *__restrict__ Phi, int n2, int St, int b,
                         double *__restrict__ J, size_t ld) {
  const size_t Nh = (size_t)n2 * St;
  const size_t total = Nh * Nh;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t row = idx / Nh, col = idx - (idx / Nh) * Nh;
    const int i = (int)(row / St), s = (int)(row % St), j = (int)(col / St), t = (int)(col % St);
    const double v = A[((size_t)b * St + s) * St + t] * Phi[(((size_t)b * St + t) * n2 + i) * n2 + j];
    J[row * ld + col] = v - (row == col ? 1.0 : 0.0);
  }
}

// Border of the hyper-time Newton matrix for the unknown frequencies (d > e), through
// Z = Gamma^-1 zbar (the paper gives this form no phase condition): column Nh + u holds
// dR/domega_{e+u} = (I (x) Gamma dR(rho)/domega Gamma^-1) zbar(2 pi), with R(rho) Gamma^-1 zbar(2 pi)
// = RGi zbar(2 pi) and d alpha_l / d omega = 2 pi k / omega_1; row Nh + u is the phase row of
// Eq. (18), [(I (x) nabla_{phi_{e+u}}) Gamma^-1 zbar(0)]^T (I (x) Gamma^-1).  One point (b = 0).
__global__ void k_ht_border(double *__restrict__ J, size_t ld, int Nh, int nu, int n2, int St, int U, int L,
                            const double *__restrict__ zT, int ldw, const double *__restrict__ zb0,
                            const double *__restrict__ RGi, const double *__restrict__ G,
                            const double *__restrict__ Gi, const int32_t *__restrict__ ktable, int dm1, int e,
                            double c_w) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Nh * nu) return;
  const int u = idx / Nh, rr = idx - u * Nh, i = rr / St, s = rr - i * St;
  double col = 0.0, row = 0.0;
  for (int l = 0; l < L; ++l) {
    const double k = (double)ktable[(size_t)l * dm1 + e + u - 1];
    if (k == 0.0) continue;
    const double *rc = RGi + (size_t)(2 * l + 1) * St, *rs = rc + St;
    const double *gc = Gi + (size_t)(2 * l + 1) * St, *gs = gc + St;
    double wc = 0.0, ws = 0.0, vc = 0.0, vs = 0.0;
    for (int t = 0; t < St; ++t) {
      const double zt = zT[(size_t)i * ldw + t], z0 = zb0[(size_t)i * St + t];
      wc += rc[t] * zt;
      ws += rs[t] * zt;
      vc += gc[t] * z0;
      vs += gs[t] * z0;
    }
    col += c_w * k * (G[(size_t)s * U + 2 * l + 1] * (-ws) + G[(size_t)s * U + 2 * l + 2] * wc);
    row += k * (vs * gc[s] - vc * gs[s]);
  }
  J[(size_t)rr * ld + Nh + u] = col;
  J[(size_t)(Nh + u) * ld + rr] = row;
  if (rr < nu) J[(size_t)(Nh + u) * ld + Nh + rr] = 0.0;
}

fse_status ht_buffers(fse_ctx *ctx) {
  const size_t St = ctx->St, U = ctx->U, B = ctx->Bmax, Nh = 2 * (size_t)ctx->n * St;
  const size_t need = B * U * St + B * St * St + B * Nh + (ctx->d - ctx->e);
  if (ctx->ht_elems < need) {
    if (ctx->ht) (void)hipFree(ctx->ht);
    ctx->ht = nullptr;
    ctx->ht_elems = 0;
    if (hipMalloc((void **)&ctx->ht, sizeof(double) * need) != hipSuccess) {
      ctx->err = "hipMalloc failed for the hyper-time buffers";
      return FSE_E_NOMEM;
    }
    ctx->ht_elems = need;
  }
  return FSE_OK;
}

}  // namespace

fse_status launch_samples_in(fse_ctx *ctx, int B, const double *zbar0) {
  const int W = B * ctx->St;
  dim3 grid((W + 127) / 128, 2 * ctx->n);
  hipLaunchKernelGGL(k_samples_in, grid, dim3(128), 0, ctx->stream, zbar0, ctx->n, ctx->St, W, ctx->Wmax,
                     ctx->qhist, ctx->u0);
  FSE_HIP(hipGetLastError());
  return FSE_OK;
}

// Residual and (J != null) Jacobian of B points, each J with leading dimension ld >= 2n S~.
static fse_status ht_system(fse_ctx *ctx, int32_t B, const double *omega, const double *zbar0, double *R,
                            double *rnorm, double *J, size_t ld) {
  if (B < 1 || B > ctx->Bmax) {
    ctx->err = "B out of range [1, max_batch]";
    return FSE_E_INVAL;
  }
  double *Phi = nullptr;
  if (J) {
    FSE_TRY(ensure_phi_buffer(ctx));
    Phi = ctx->PhiQU;
  }
  FSE_TRY(ht_buffers(ctx));
  ctx->samples_in = true;
  const fse_status st = integrate_points(ctx, B, omega, zbar0, nullptr, Phi);
  ctx->samples_in = false;
  FSE_TRY(st);
  const int U = ctx->U, St = ctx->St, n2 = 2 * ctx->n;
  const size_t Nh = (size_t)n2 * St;
  double *RGi = ctx->ht, *A = RGi + (size_t)ctx->Bmax * U * St;
  const int Lm = ctx->L > 0 ? ctx->L : 1;
  hipLaunchKernelGGL(k_ht_rgi, dim3((U * St + 255) / 256, B), dim3(256), 0, ctx->stream, ctx->Gi_d, ctx->rot_d, U,
                     St, Lm, RGi);
  hipLaunchKernelGGL(k_ht_A, dim3((St * St + 255) / 256, B), dim3(256), 0, ctx->stream, ctx->G_d, RGi, U, St, A);
  const size_t tot = Nh * B;
  hipLaunchKernelGGL(k_ht_residual, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, ctx->zTw,
                     ctx->Wmax, A, zbar0, n2, St, B, R);
  FSE_HIP(hipGetLastError());
  if (rnorm)
    for (int b = 0; b < B; ++b) FSE_TRY(launch_norm(ctx, R + (size_t)b * Nh, Nh, rnorm + b));
  if (J) {
    const size_t total = Nh * Nh;
    const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 1u << 20);
    for (int b = 0; b < B; ++b)
      hipLaunchKernelGGL(k_ht_jac, dim3(blocks), dim3(256), 0, ctx->stream, A, Phi, n2, St, b, J + (size_t)b * ld * ld,
                         ld);
    FSE_HIP(hipGetLastError());
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

extern "C" {

fse_status fse_hypertime_residual_jacobian(fse_ctx *ctx, int32_t B, const double *omega, const double *zbar0,
                                           double *R, double *rnorm, double *J) {
  if (!ctx || !omega || !zbar0 || !R) return FSE_E_INVAL;
  return ht_system(ctx, B, omega, zbar0, R, rnorm, J, 2 * (size_t)ctx->n * ctx->St);
}

fse_status fse_hypertime_newton_step(fse_ctx *ctx, double *omega, double *zbar0, double *res_norm) {
  if (!ctx || !omega || !zbar0) return FSE_E_INVAL;
  const size_t Nh = 2 * (size_t)ctx->n * ctx->St;
  const int nu = ctx->d - ctx->e;
  const size_t Nb = Nh + nu;
  if (Nb > (size_t)INT32_MAX / 2) {
    ctx->err = "too many hyper-time unknowns for the dense Newton step";
    return FSE_E_UNSUPPORTED;
  }
  FSE_TRY(ht_buffers(ctx));
  FSE_TRY(ensure_dense_matrix(ctx, Nb));
  const double *RGi = ctx->ht;
  double *R = ctx->ht + (size_t)ctx->Bmax * ctx->U * ctx->St + (size_t)ctx->Bmax * ctx->St * ctx->St;
  double rn = 0.0;
  FSE_TRY(ht_system(ctx, 1, omega, zbar0, R, &rn, ctx->Jw, Nb));
  if (res_norm) *res_norm = rn;
  if (nu > 0) {
    hipLaunchKernelGGL(k_ht_border, dim3((unsigned)((Nh * nu + 255) / 256)), dim3(256), 0, ctx->stream, ctx->Jw, Nb,
                       (int)Nh, nu, 2 * ctx->n, ctx->St, ctx->U, ctx->L, ctx->zTw, ctx->Wmax, zbar0, RGi, ctx->G_d,
                       ctx->Gi_d, ctx->ktable_d, ctx->d - 1, ctx->e, 2.0 * M_PI / omega[0]);
    FSE_HIP(hipGetLastError());
    FSE_HIP(hipMemsetAsync(R + Nh, 0, sizeof(double) * nu, ctx->stream));
  }
  FSE_TRY(dense_lu_solve(ctx, ctx->Jw, (int)Nb, R));
  FSE_TRY(launch_axpy(ctx, (int)Nh, -1.0, R, zbar0));
  if (nu > 0) {
    std::vector<double> dw(nu);
    FSE_HIP(hipMemcpyAsync(dw.data(), R + Nh, sizeof(double) * nu, hipMemcpyDeviceToHost, ctx->stream));
    FSE_HIP(hipStreamSynchronize(ctx->stream));
    for (int u = 0; u < nu; ++u) omega[ctx->e + u] -= dw[u];
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

}  // extern "C"
