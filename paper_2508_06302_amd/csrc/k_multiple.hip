// Multiple FSE-Shooting on gfx950: the period of phi_1 cut into M segments (the paper's
// first recommendation for future work, read as classical multiple shooting of Sec. 3).
//
// Unknowns: the sections Z^(m) [2n][U~] of the torus at phi_1 = 2 pi m / M.  Segment m is a
// batch point: its trajectories start on section m at the grid phases (inverse DFT, Eq. 20),
// with the forcing of frequency 1 at phase 2 pi m / M, and run S1 / M steps.  Residual and
// Jacobian (unknowns [Z^(0); ...; Z^(M-1)]):
//     R_m = (I (x) R(rho / M)) Gamma^-1 zbar^(m) - Z^((m + 1) mod M),
//     dR_m / dZ^(m) = Eq. (22) operator of segment m without -I,  dR_m / dZ^(m+1) = -I.
// M = 1 is FSE-Shooting.  d = e only.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fse_internal.h"

namespace {

// J (row-major, MN x MN, diagonal blocks from the single-segment Jacobian, which carries -I):
// +I on the diagonal blocks, -I on the blocks (m, m + 1 mod M); one thread per row.
__global__ void k_mult_blocks(double *__restrict__ J, int N, int M, size_t ld) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int m = idx / N, i = idx - (idx / N) * N;
  const size_t row = (size_t)m * N + i;
  J[row * ld + row] += 1.0;
  J[row * ld + (size_t)((m + 1) % M) * N + i] -= 1.0;
}

// Border of the multiple-shooting Newton matrix for the unknown base frequencies (d > e):
// column M N + u holds dR_m/domega_{e+u} = (I (x) dR(rho/M)/domega) Gamma^-1 zbar^(m), with
// R(rho/M) Gamma^-1 zbar^(m) = R_m + Z^(m+1) and d alpha_l / d omega_{e+u} = 2 pi k / (M omega_1);
// row M N + u is the phase row of Eq. (18) on section 0 (zero over the other sections, which
// the caller has cleared).
__global__ void k_mult_border(double *__restrict__ J, size_t ld, int M, int N, int nu, const double *__restrict__ R,
                              const double *__restrict__ Zs, const int32_t *__restrict__ ktable, int dm1, int e,
                              double c_w, int U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int MN = M * N;
  if (idx >= MN * nu) return;
  const int u = idx / MN, rr = idx - u * MN, m = rr / N, r = rr - m * N;
  const int a = r % U, base = r - a;
  const double *Rm = R + (size_t)m * N, *Zn = Zs + (size_t)((m + 1) % M) * N;
  double dr = 0.0, pr = 0.0;
  if (a > 0) {
    const double k = (double)ktable[(size_t)((a - 1) / 2) * dm1 + e + u - 1];
    if (a & 1) {  // cos coefficient of the pair
      dr = -c_w * k * (Rm[base + a + 1] + Zn[base + a + 1]);
      pr = k * Zs[base + a + 1];
    } else {      // sin coefficient
      dr = c_w * k * (Rm[base + a - 1] + Zn[base + a - 1]);
      pr = -k * Zs[base + a - 1];
    }
  }
  J[(size_t)rr * ld + MN + u] = dr;
  if (m == 0) J[(size_t)(MN + u) * ld + r] = pr;
}

fse_status mult_buffers(fse_ctx *ctx, int M) {
  const size_t N = 2 * (size_t)ctx->n * ctx->U, need = 2 * (size_t)M * N + (ctx->d - ctx->e);
  if (ctx->mult_elems < need) {
    if (ctx->mult) (void)hipFree(ctx->mult);
    ctx->mult = nullptr;
    ctx->mult_elems = 0;
    if (hipMalloc((void **)&ctx->mult, sizeof(double) * need) != hipSuccess) {
      ctx->err = "hipMalloc failed for the multiple-shooting buffers";
      return FSE_E_NOMEM;
    }
    ctx->mult_elems = need;
  }
  return FSE_OK;
}

fse_status mult_check(fse_ctx *ctx, int M) {
  if (M < 1 || M > ctx->Bmax) {
    ctx->err = "the number of segments must be in [1, max_batch]";
    return FSE_E_INVAL;
  }
  if (ctx->S1 % M != 0) {
    ctx->err = "S1 must be a multiple of the number of segments";
    return FSE_E_INVAL;
  }
  return FSE_OK;
}

// Residual (and the block-cyclic Jacobian into J with leading dimension ld >= M N) of the
// M segments at (omega, Zs).
fse_status mult_system(fse_ctx *ctx, int M, const double *omega, const double *Zs, double *R, double *rnorm,
                       double *J, size_t ld) {
  const size_t N = 2 * (size_t)ctx->n * ctx->U;
  FSE_TRY(mult_buffers(ctx, M));
  double *Phi = nullptr;
  if (J) {
    FSE_TRY(ensure_phi_buffer(ctx));
    Phi = ctx->PhiQU;
  }
  // every segment is a batch point with the same frequencies
  std::vector<double> om((size_t)M * ctx->d);
  for (int m = 0; m < M; ++m)
    for (int j = 0; j < ctx->d; ++j) om[(size_t)m * ctx->d + j] = omega[j];
  ctx->seg_steps = ctx->S1 / M;
  ctx->seg_phase = 2.0 * M_PI / M;
  const fse_status st = integrate_points(ctx, M, om.data(), Zs, nullptr, Phi);
  ctx->seg_steps = 0;
  ctx->seg_phase = 0.0;
  FSE_TRY(st);
  // rotation by rho / M for every segment
  const int Lm = std::max(ctx->L, 1), dm1 = ctx->d - 1;
  std::vector<double> rot((size_t)M * Lm, 0.0);
  for (int l = 0; l < ctx->L; ++l) {
    double a = 0.0;
    for (int j = 0; j < dm1; ++j) a += (double)ctx->ktable[(size_t)l * dm1 + j] * (omega[1 + j] / omega[0]);
    for (int m = 0; m < M; ++m) rot[(size_t)m * Lm + l] = 2.0 * M_PI * a / M;
  }
  FSE_HIP(hipMemcpyAsync(ctx->rot_d, rot.data(), sizeof(double) * rot.size(), hipMemcpyHostToDevice, ctx->stream));
  // the section each segment must reach: Z^((m + 1) mod M)
  double *Znext = ctx->mult;
  for (int m = 0; m < M; ++m)
    FSE_HIP(hipMemcpyAsync(Znext + (size_t)m * N, Zs + (size_t)((m + 1) % M) * N, sizeof(double) * N,
                           hipMemcpyDeviceToDevice, ctx->stream));
  FSE_TRY(launch_dft(ctx, M, ctx->zTw, Znext, R));
  if (rnorm) FSE_TRY(launch_norm(ctx, R, (size_t)M * N, rnorm));
  if (J) {
    FSE_HIP(hipMemsetAsync(J, 0, sizeof(double) * ld * ld, ctx->stream));
    const size_t phi_seg = (size_t)ctx->St * 4 * ctx->n * ctx->n;
    for (int m = 0; m < M; ++m)
      FSE_TRY(launch_jacobian(ctx, 1, Phi + (size_t)m * phi_seg, J + (size_t)m * N * ld + (size_t)m * N, ld));
    hipLaunchKernelGGL(k_mult_blocks, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, ctx->stream, J, (int)N,
                       M, ld);
    FSE_HIP(hipGetLastError());
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

}  // namespace

extern "C" {

fse_status fse_multiple_residual_jacobian(fse_ctx *ctx, int32_t M, const double *omega, const double *Zs,
                                          double *R, double *rnorm, double *J) {
  if (!ctx || !omega || !Zs || !R) return FSE_E_INVAL;
  FSE_TRY(mult_check(ctx, M));
  const size_t N = 2 * (size_t)ctx->n * ctx->U;
  if ((size_t)M * N > (size_t)INT32_MAX / 2) {
    ctx->err = "too many unknowns";
    return FSE_E_UNSUPPORTED;
  }
  return mult_system(ctx, M, omega, Zs, R, rnorm, J, (size_t)M * N);
}

fse_status fse_multiple_newton_step(fse_ctx *ctx, int32_t M, double *omega, double *Zs, double *res_norm) {
  if (!ctx || !omega || !Zs) return FSE_E_INVAL;
  FSE_TRY(mult_check(ctx, M));
  const size_t N = 2 * (size_t)ctx->n * ctx->U, NM = (size_t)M * N;
  const int nu = ctx->d - ctx->e;
  const size_t Nb = NM + nu;
  if (Nb > (size_t)INT32_MAX / 2) {
    ctx->err = "too many unknowns for the dense Newton step";
    return FSE_E_UNSUPPORTED;
  }
  FSE_TRY(mult_buffers(ctx, M));
  FSE_TRY(ensure_dense_matrix(ctx, Nb));
  double *R = ctx->mult + NM;  // [M N + nu]: residuals, then the phase-row zeros
  double rn = 0.0;
  FSE_TRY(mult_system(ctx, M, omega, Zs, R, &rn, ctx->Jw, Nb));
  if (res_norm) *res_norm = rn;
  if (nu > 0) {
    hipLaunchKernelGGL(k_mult_border, dim3((unsigned)((NM * nu + 255) / 256)), dim3(256), 0, ctx->stream, ctx->Jw,
                       Nb, M, (int)N, nu, R, Zs, ctx->ktable_d, ctx->d - 1, ctx->e, 2.0 * M_PI / (M * omega[0]),
                       ctx->U);
    FSE_HIP(hipGetLastError());
    FSE_HIP(hipMemsetAsync(R + NM, 0, sizeof(double) * nu, ctx->stream));
  }
  FSE_TRY(dense_lu_solve(ctx, ctx->Jw, (int)Nb, R));
  FSE_TRY(launch_axpy(ctx, (int)NM, -1.0, R, Zs));
  if (nu > 0) {
    std::vector<double> dw(nu);
    FSE_HIP(hipMemcpyAsync(dw.data(), R + NM, sizeof(double) * nu, hipMemcpyDeviceToHost, ctx->stream));
    FSE_HIP(hipStreamSynchronize(ctx->stream));
    for (int u = 0; u < nu; ++u) omega[ctx->e + u] -= dw[u];
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

}  // extern "C"
