// Matrix-free Newton-Krylov for the shooting problem (Sec. 3.3 step 6 with Eq. 22 applied to
// vectors) on gfx950.
//
// The Jacobian of Eq. (22) is never formed: with the trajectory sensitivities Phi_s of the
// last evaluation,
//     J v = (I (x) R(rho) Gamma^-1) blkdiag_s(Phi_s) (I (x) Gamma) v - v,
// i.e. k_gamma_expand (coefficients -> samples), k_phi_apply (one 2n x 2n matrix-vector
// product per trajectory, bound by reading Phi from HBM) and the DFT + rotation kernel of the
// residual.  The Newton correction solves J dZ = -R by restarted GMRES with right
// preconditioning, classical Gram-Schmidt applied twice for the Arnoldi basis on the GPU and
// Givens rotations on the small Hessenberg matrix on the host.
//
// Preconditioner: P = Phi_bar (x) R(rho) - I, Phi_bar the mean of Phi_s over the trajectories.
// For a linear system every Phi_s is the same matrix and P = J.  R(rho) is block-diagonal
// per harmonic, so P is one 2n x 2n block (zero harmonic) and one 4n x 4n block per harmonic
// pair, [[c Phi_bar - I, -s Phi_bar], [s Phi_bar, c Phi_bar - I]] with (c, s) the rotation of
// that pair; each block is factored once per Newton step with the dense LU.
#include <cmath>
#include <vector>

#include <mutex>

#include "fse_internal.h"

// Fixed device scratch of fse_jacobian_apply_noalloc (callers that cannot allocate): one copy per
// GPU for the life of the process.  Host code never uses the symbol's name as a device address;
// fse_init_torus takes the address on each device once (noalloc_setup) and kernels receive it.
static __device__ __align__(256) double scratch[kNoAllocScratch];
static double *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

fse_status noalloc_setup(fse_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) {
    ctx->err = "device index beyond the no-allocation scratch table";
    return FSE_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[ctx->device]) return FSE_OK;
  void *p = nullptr;
  FSE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch_ptr[ctx->device] = static_cast<double *>(p);
  return FSE_OK;
}

double *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

namespace {

// x[j][w] = sum_m Gamma[w][m] v[j][m], w < S~ (one point)
__global__ void k_gamma_expand(const double *__restrict__ v, const double *__restrict__ G, int n2, int U, int St,
                               int ldw, double *__restrict__ x) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (w >= St || j >= n2) return;
  const double *g = G + (size_t)w * U;
  const double *vj = v + (size_t)j * U;
  double acc = 0.0;
  for (int m = 0; m < U; ++m) acc += g[m] * vj[m];
  x[(size_t)j * ldw + w] = acc;
}

// y[i][w] = sum_j Phi_w[i][j] x[j][w]: work-group (w, row block); x_w staged in LDS, one
// wave per row with the lanes along the (contiguous) row of Phi_w.
constexpr int kPhiRows = 32;

__global__ __launch_bounds__(256) void k_phi_apply(const double *__restrict__ Phi, const double *__restrict__ x,
                                                   int n2, int ldw, double *__restrict__ y) {
  extern __shared__ double xs[];
  const int w = blockIdx.x, i0 = blockIdx.y * kPhiRows;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < n2; j += blockDim.x) xs[j] = x[(size_t)j * ldw + w];
  __syncthreads();
  const int i1 = min(i0 + kPhiRows, n2);
  for (int i = i0 + wave; i < i1; i += 4) {
    const double *row = Phi + ((size_t)w * n2 + i) * n2;
    double acc = 0.0;
    for (int j = lane; j < n2; j += 64) acc += row[j] * xs[j];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) y[(size_t)i * ldw + w] = acc;
  }
}

// Phi_bar[i][j] = (1 / S~) sum_s Phi_s[i][j]
__global__ void k_phi_mean(const double *__restrict__ Phi, int n2, int St, double *__restrict__ Pbar) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)n2 * n2;
  if (idx >= nn) return;
  double acc = 0.0;
  for (int s = 0; s < St; ++s) acc += Phi[(size_t)s * nn + idx];
  Pbar[idx] = acc / (double)St;
}

// Preconditioner blocks, row-major: block 0 = Phi_bar - I (n2 x n2) at offset 0; block l >= 1
// (harmonic pair l, rotation angle alpha_l = rot[l - 1]) = [[c P - I, -s P], [s P, c P - I]]
// (2 n2 x 2 n2) at offset n2^2 + (l - 1) (2 n2)^2.
__global__ void k_pc_blocks(const double *__restrict__ Pbar, const double *__restrict__ rot, int n2, int L,
                            double *__restrict__ blocks) {
  const int l = blockIdx.y;
  const size_t m = l == 0 ? (size_t)n2 : 2 * (size_t)n2;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l > L || idx >= m * m) return;
  const size_t r = idx / m, c = idx % m;
  double v;
  if (l == 0) {
    v = Pbar[r * n2 + c] - (r == c ? 1.0 : 0.0);
  } else {
    const double a = rot[l - 1], cs = cos(a), sn = sin(a);
    const bool rs = r >= (size_t)n2, csd = c >= (size_t)n2;
    const double p = Pbar[(r % n2) * n2 + (c % n2)];
    const double f = (rs == csd) ? cs : (rs ? sn : -sn);
    v = f * p - (r == c ? 1.0 : 0.0);
  }
  const size_t off = l == 0 ? 0 : (size_t)n2 * n2 + (size_t)(l - 1) * 4 * n2 * n2;
  blocks[off + idx] = v;
}

// Coefficient layout v[i][a] (a < U; a = 0 zero harmonic, a = 2l - 1 / 2l the cos / sin of
// pair l) <-> block layout: block 0 holds v[i][0]; block l holds v[i][2l - 1], then v[i][2l].
__global__ void k_pc_gather(double *__restrict__ v, int n2, int U, double *__restrict__ bv, int dir) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n2 * U) return;
  const int i = idx / U, a = idx - (idx / U) * U;
  int pos;
  if (a == 0) {
    pos = i;
  } else {
    const int l = (a + 1) / 2;
    pos = n2 + (l - 1) * 2 * n2 + ((a & 1) ? i : n2 + i);
  }
  if (dir == 0)
    bv[pos] = v[idx];
  else
    v[idx] = bv[pos];
}

// h[j] = <V_j, w> for j < k (one work-group per j)
__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ V, size_t ldv, const double *__restrict__ w,
                                              int N, double *__restrict__ h) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const double *vj = V + (size_t)j * ldv;
  double acc = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) acc += vj[i] * w[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) h[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w += alpha sum_{j < k} h[j] V_j
__global__ void k_vcomb(const double *__restrict__ V, size_t ldv, int k, const double *__restrict__ h, int N,
                        double alpha, double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += h[j] * V[(size_t)j * ldv + i];
  w[i] += alpha * acc;
}

__global__ void k_scale(int N, double a, const double *__restrict__ x, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = a * x[i];
}

// out[r] += sum_u Bc[u][r] w[u] (r < N)
__global__ void k_add_cols(const double *__restrict__ Bc, int N, int nu, const double *__restrict__ w,
                           double *__restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  double acc = out[r];
  for (int u = 0; u < nu; ++u) acc += Bc[(size_t)u * N + r] * w[u];
  out[r] = acc;
}

// Border of the Newton matrix for the unknown base frequencies omega_{e+1..d} at (Z0, R):
// Bc[u] = dR/domega_{e+u} (rotation term of Eqs. 23-24, d alpha_l / d omega = 2 pi k / omega_1,
// applied to R + Z0 = R(rho) Z(2 pi)), Pr[u] = (I (x) nabla_{phi_{e+u}}) Z0 (the phase row of
// Eq. 18 with Z* = dZ).
__global__ void k_kr_border(double *__restrict__ Bc, double *__restrict__ Pr, int N, int nu,
                            const double *__restrict__ R, const double *__restrict__ Z0,
                            const int32_t *__restrict__ ktable, int dm1, int e, double two_pi_over_w1, int U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nu) return;
  const int u = idx / N, r = idx - u * N;
  const int a = r % U, base = r - a;
  double dr = 0.0, pr = 0.0;
  if (a > 0) {
    const double k = (double)ktable[(size_t)((a - 1) / 2) * dm1 + e + u - 1];
    if (a & 1) {  // cos coefficient of the pair
      dr = -two_pi_over_w1 * k * (R[base + a + 1] + Z0[base + a + 1]);
      pr = k * Z0[base + a + 1];
    } else {      // sin coefficient
      dr = two_pi_over_w1 * k * (R[base + a - 1] + Z0[base + a - 1]);
      pr = -k * Z0[base + a - 1];
    }
  }
  Bc[(size_t)u * N + r] = dr;
  Pr[(size_t)u * N + r] = pr;
}

// Unknowns [Z(0); omega_u] (Nb = N + nu entries; nu = d - e unknown base frequencies): the
// Newton matrix is [[J, dR/domega_u], [phase rows, 0]] (Eqs. 17-18, 23-24).  Bc holds the
// columns dR/domega_u and Pr the phase rows, [nu][N] each.
struct Krylov {
  fse_ctx *ctx;
  int N, Nb, nu, n2, U, L;
  size_t ldv;
  double *V, *w, *z, *u, *r, *x, *b, *h, *bv, *xs, *ys, *Pbar, *Bc, *Pr, *blocks;
  int32_t *piv;
};

fse_status kr_alloc(fse_ctx *ctx, int restart) {
  const size_t N = (size_t)2 * ctx->n * ctx->U, n2 = 2 * (size_t)ctx->n;
  const size_t L = (size_t)ctx->L;
  const size_t blk = n2 * n2 + L * 4 * n2 * n2;
  const size_t Nb = N + (size_t)(ctx->d - ctx->e);
  const size_t need = (size_t)(restart + 1) * Nb + 6 * Nb + (restart + 2) + Nb + 2 * n2 * ctx->Wmax + n2 * n2 +
                      2 * (Nb - N) * N + blk;
  if (ctx->kr_elems < need) {
    if (ctx->kr) (void)hipFree(ctx->kr);
    if (ctx->kr_piv) (void)hipFree(ctx->kr_piv);
    ctx->kr = nullptr;
    ctx->kr_piv = nullptr;
    ctx->kr_elems = 0;
    ctx->pc_ready = false;
    if (hipMalloc((void **)&ctx->kr, sizeof(double) * need) != hipSuccess ||
        hipMalloc((void **)&ctx->kr_piv, sizeof(int32_t) * (n2 + 2 * L * n2)) != hipSuccess) {
      ctx->err = "hipMalloc failed for the Krylov workspace";
      return FSE_E_NOMEM;
    }
    ctx->kr_elems = need;
  }
  return FSE_OK;
}

Krylov kr_view(fse_ctx *ctx, int restart) {
  Krylov k;
  k.ctx = ctx;
  k.N = 2 * ctx->n * ctx->U;
  k.nu = ctx->d - ctx->e;
  k.Nb = k.N + k.nu;
  k.n2 = 2 * ctx->n;
  k.U = ctx->U;
  k.L = ctx->L;
  k.ldv = (size_t)k.Nb;
  double *p = ctx->kr;
  k.V = p;
  p += (size_t)(restart + 1) * k.Nb;
  k.w = p;
  p += k.Nb;
  k.z = p;
  p += k.Nb;
  k.u = p;
  p += k.Nb;
  k.r = p;
  p += k.Nb;
  k.x = p;
  p += k.Nb;
  k.b = p;
  p += k.Nb;
  k.h = p;
  p += restart + 2;
  k.bv = p;
  p += k.Nb;
  k.xs = p;
  p += (size_t)k.n2 * ctx->Wmax;
  k.ys = p;
  p += (size_t)k.n2 * ctx->Wmax;
  k.Pbar = p;
  p += (size_t)k.n2 * k.n2;
  k.Bc = p;
  p += (size_t)k.nu * k.N;
  k.Pr = p;
  p += (size_t)k.nu * k.N;
  k.blocks = p;
  k.piv = ctx->kr_piv;
  return k;
}

// out = J v with the stored sensitivities (ctx->PhiQU) and the rotation of the same evaluation
// (ctx->rot_mf);
// with unknown frequencies, out = [J v_Z + dR/domega_u v_w; phase rows . v_Z]
fse_status kr_matvec(const Krylov &k, const double *v, double *out) {
  fse_ctx *ctx = k.ctx;
  const int St = ctx->St, W = ctx->Wmax;
  hipLaunchKernelGGL(k_gamma_expand, dim3((St + 63) / 64, k.n2), dim3(64), 0, ctx->stream, v, ctx->G_d, k.n2, k.U,
                     St, W, k.xs);
  hipLaunchKernelGGL(k_phi_apply, dim3(St, (k.n2 + kPhiRows - 1) / kPhiRows), dim3(256), sizeof(double) * k.n2,
                     ctx->stream, ctx->PhiQU, k.xs, k.n2, W, k.ys);
  FSE_HIP(hipGetLastError());
  FSE_TRY(launch_dft(ctx, 1, k.ys, v, out, ctx->rot_mf));
  if (k.nu > 0) {
    hipLaunchKernelGGL(k_add_cols, dim3((k.N + 255) / 256), dim3(256), 0, ctx->stream, k.Bc, k.N, k.nu, v + k.N,
                       out);
    hipLaunchKernelGGL(k_dots, dim3(k.nu), dim3(256), 0, ctx->stream, k.Pr, (size_t)k.N, v, k.N, out + k.N);
    FSE_HIP(hipGetLastError());
  }
  return FSE_OK;
}

size_t block_off(const Krylov &k, int l) {
  return l == 0 ? 0 : (size_t)k.n2 * k.n2 + (size_t)(l - 1) * 4 * k.n2 * k.n2;
}
size_t vec_off(const Krylov &k, int l) { return l == 0 ? 0 : (size_t)k.n2 + (size_t)(l - 1) * 2 * k.n2; }

fse_status kr_precond_build(const Krylov &k) {
  fse_ctx *ctx = k.ctx;
  const size_t nn = (size_t)k.n2 * k.n2;
  hipLaunchKernelGGL(k_phi_mean, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, ctx->stream, ctx->PhiQU, k.n2,
                     ctx->St, k.Pbar);
  hipLaunchKernelGGL(k_pc_blocks, dim3((unsigned)((4 * nn + 255) / 256), k.L + 1), dim3(256), 0, ctx->stream,
                     k.Pbar, ctx->rot_mf, k.n2, k.L, k.blocks);
  FSE_HIP(hipGetLastError());
  for (int l = 0; l <= k.L; ++l) {
    const int m = l == 0 ? k.n2 : 2 * k.n2;
    FSE_TRY(dense_lu_factor(ctx, k.blocks + block_off(k, l), m, k.piv + vec_off(k, l)));
  }
  ctx->pc_ready = true;
  return FSE_OK;
}

// out = P^-1 v (out may alias v)
fse_status kr_precond_apply(const Krylov &k, const double *v, double *out) {
  fse_ctx *ctx = k.ctx;
  const int nth = 256, nbk = (k.N + nth - 1) / nth;
  hipLaunchKernelGGL(k_pc_gather, dim3(nbk), dim3(nth), 0, ctx->stream, const_cast<double *>(v), k.n2, k.U, k.bv,
                     0);
  FSE_HIP(hipGetLastError());
  // the zero-harmonic block, then the L harmonic-pair blocks (one size, evenly spaced) as a batch
  FSE_TRY(dense_lu_apply(ctx, k.blocks, k.n2, k.piv, k.bv));
  if (k.L > 0) {
    const size_t m = 2 * (size_t)k.n2;
    FSE_TRY(dense_lu_apply_batched(ctx, k.blocks + block_off(k, 1), m * m, (int)m, k.piv + vec_off(k, 1), m,
                                   k.bv + vec_off(k, 1), m, k.L));
  }
  hipLaunchKernelGGL(k_pc_gather, dim3(nbk), dim3(nth), 0, ctx->stream, out, k.n2, k.U, k.bv, 1);
  FSE_HIP(hipGetLastError());
  // the frequency unknowns are not preconditioned
  if (k.nu > 0 && out != v)
    FSE_HIP(hipMemcpyAsync(out + k.N, v + k.N, sizeof(double) * k.nu, hipMemcpyDeviceToDevice, ctx->stream));
  return FSE_OK;
}

fse_status kr_norm(const Krylov &k, const double *v, double *out) { return launch_norm(k.ctx, v, (size_t)k.Nb, out); }

// Right-preconditioned restarted GMRES for J x = b (b device [N]); x returned in k.x.
fse_status kr_gmres(const Krylov &k, const double *b, bool precond, double rtol, int restart, int maxit, int *its_out,
                    double *rel_out) {
  fse_ctx *ctx = k.ctx;
  const int N = k.Nb, nth = 256, nbk = (N + nth - 1) / nth;  // every vector has the Nb unknowns
  double nb = 0.0;
  FSE_TRY(kr_norm(k, b, &nb));
  FSE_HIP(hipMemsetAsync(k.x, 0, sizeof(double) * N, ctx->stream));
  *its_out = 0;
  *rel_out = 0.0;
  if (!(nb > 0.0)) return FSE_OK;
  std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), hh(restart + 2),
      hh2(restart + 2), y(restart);
  int its = 0;
  while (true) {
    // r = b - J x
    FSE_TRY(kr_matvec(k, k.x, k.r));
    FSE_TRY(launch_axpby(ctx, N, 1.0, b, -1.0, k.r, k.r));
    double beta = 0.0;
    FSE_TRY(kr_norm(k, k.r, &beta));
    *rel_out = beta / nb;
    if (beta <= rtol * nb || its >= maxit) break;
    if (!std::isfinite(beta)) {
      ctx->err = "GMRES residual is not finite";
      return FSE_E_NAN;
    }
    hipLaunchKernelGGL(k_scale, dim3(nbk), dim3(nth), 0, ctx->stream, N, 1.0 / beta, k.r, k.V);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int m = 0;
    for (int j = 0; j < restart; ++j) {
      double *vj = k.V + (size_t)j * k.ldv;
      if (precond) {
        FSE_TRY(kr_precond_apply(k, vj, k.z));
        FSE_TRY(kr_matvec(k, k.z, k.w));
      } else {
        FSE_TRY(kr_matvec(k, vj, k.w));
      }
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_dots, dim3(j + 1), dim3(256), 0, ctx->stream, k.V, k.ldv, k.w, N, k.h);
        hipLaunchKernelGGL(k_vcomb, dim3(nbk), dim3(nth), 0, ctx->stream, k.V, k.ldv, j + 1, k.h, N, -1.0, k.w);
        FSE_HIP(hipGetLastError());
        FSE_HIP(hipMemcpyAsync(pass == 0 ? hh.data() : hh2.data(), k.h, sizeof(double) * (j + 1),
                               hipMemcpyDeviceToHost, ctx->stream));
      }
      double hn = 0.0;
      FSE_TRY(kr_norm(k, k.w, &hn));  // synchronises the stream, so hh and hh2 are in place
      for (int i = 0; i <= j; ++i) H[(size_t)i * restart + j] = hh[i] + hh2[i];
      H[(size_t)(j + 1) * restart + j] = hn;
      hipLaunchKernelGGL(k_scale, dim3(nbk), dim3(nth), 0, ctx->stream, N, hn > 0.0 ? 1.0 / hn : 0.0, k.w,
                         k.V + (size_t)(j + 1) * k.ldv);
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * restart + j], c = H[(size_t)(i + 1) * restart + j];
        H[(size_t)i * restart + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * restart + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * restart + j], c = H[(size_t)(j + 1) * restart + j];
      const double den = std::hypot(a, c);
      cs[j] = den > 0.0 ? a / den : 1.0;
      sn[j] = den > 0.0 ? c / den : 0.0;
      H[(size_t)j * restart + j] = den;
      H[(size_t)(j + 1) * restart + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      m = j + 1;
      if (std::fabs(g[j + 1]) <= rtol * nb || its >= maxit || !(hn > 0.0)) break;
    }
    // y = H^-1 g (upper triangular), u = V y, x += P^-1 u
    for (int i = m - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < m; ++c) acc -= H[(size_t)i * restart + c] * y[c];
      y[i] = acc / H[(size_t)i * restart + i];
    }
    FSE_HIP(hipMemcpyAsync(k.h, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, ctx->stream));
    FSE_HIP(hipMemsetAsync(k.u, 0, sizeof(double) * N, ctx->stream));
    hipLaunchKernelGGL(k_vcomb, dim3(nbk), dim3(nth), 0, ctx->stream, k.V, k.ldv, m, k.h, N, 1.0, k.u);
    FSE_HIP(hipGetLastError());
    if (precond) FSE_TRY(kr_precond_apply(k, k.u, k.u));
    FSE_TRY(launch_axpby(ctx, N, 1.0, k.x, 1.0, k.u, k.x));
    FSE_HIP(hipStreamSynchronize(ctx->stream));  // y stays valid until the copy is done
  }
  *its_out = its;
  return FSE_OK;
}

// Residual and sensitivities at (omega, Z0) for the matrix-free Jacobian (one point).
fse_status kr_evaluate(fse_ctx *ctx, const double *omega, const double *Z0, double *R, double *rn) {
  FSE_TRY(ensure_phi_buffer(ctx));
  FSE_TRY(integrate_points(ctx, 1, omega, Z0, nullptr, ctx->PhiQU));
  FSE_HIP(hipMemcpyAsync(ctx->rot_mf, ctx->rot_d, sizeof(double) * std::max(ctx->L, 1), hipMemcpyDeviceToDevice,
                         ctx->stream));
  FSE_TRY(launch_dft_residual(ctx, 1, Z0, R));
  FSE_TRY(launch_norms(ctx, 1, R, rn));
  ctx->mf_ready = true;
  ctx->mf_stored = true;
  ctx->pc_ready = false;
  return FSE_OK;
}

}  // namespace

extern "C" {

fse_status fse_shooting_residual_matfree(fse_ctx *ctx, const double *omega, const double *Z0, double *R,
                                         double *rnorm) {
  if (!ctx || !omega || !Z0 || !R) return FSE_E_INVAL;
  ctx->mf_ready = false;
  double rn = 0.0;
  FSE_TRY(kr_evaluate(ctx, omega, Z0, R, &rn));
  if (rnorm) *rnorm = rn;
  return FSE_OK;
}

fse_status fse_jacobian_apply(fse_ctx *ctx, const double *v, double *Jv) {
  if (!ctx || !v || !Jv) return FSE_E_INVAL;
  if (!ctx->mf_ready) {
    ctx->err = "no sensitivities: call fse_shooting_residual_matfree first";
    return FSE_E_INVAL;
  }
  FSE_TRY(kr_alloc(ctx, 1));
  Krylov k = kr_view(ctx, 1);
  k.nu = 0;  // J alone: v and Jv hold 2nU entries, without the frequency border
  FSE_TRY(kr_matvec(k, v, Jv));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_jacobian_apply_noalloc(fse_ctx *ctx, const double *v, double *Jv) {
  if (!ctx || !v || !Jv) return FSE_E_INVAL;
  if (!ctx->mf_ready) {
    ctx->err = "no sensitivities: call fse_shooting_residual_matfree first";
    return FSE_E_INVAL;
  }
  const size_t n2 = 2 * (size_t)ctx->n, W = ctx->Wmax;
  if (2 * n2 * W > kNoAllocScratch) {
    ctx->err = "fse_jacobian_apply_noalloc: 2 x 2n x (trajectories) = " + std::to_string(2 * n2 * W) +
               " doubles exceed the fixed scratch of " + std::to_string(kNoAllocScratch) + " doubles";
    return FSE_E_UNSUPPORTED;
  }
  double *base = noalloc_scratch(ctx->device);
  if (!base) {
    ctx->err = "fse_jacobian_apply_noalloc: the scratch address of this device was not set up by fse_init_torus";
    return FSE_E_DEVICE;
  }
  // (I (x) Gamma) v -> xs, Phi_s x_s -> ys (both [2n][Wmax] in the scratch), DFT + rotation - v
  double *xs = base, *ys = base + n2 * W;
  const int St = ctx->St;
  hipLaunchKernelGGL(k_gamma_expand, dim3((St + 63) / 64, (unsigned)n2), dim3(64), 0, ctx->stream, v, ctx->G_d,
                     (int)n2, ctx->U, St, (int)W, xs);
  hipLaunchKernelGGL(k_phi_apply, dim3(St, (unsigned)((n2 + kPhiRows - 1) / kPhiRows)), dim3(256),
                     sizeof(double) * n2, ctx->stream, ctx->PhiQU, xs, (int)n2, (int)W, ys);
  FSE_HIP(hipGetLastError());
  FSE_TRY(launch_dft(ctx, 1, ys, v, Jv, ctx->rot_mf));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_newton_krylov_step(fse_ctx *ctx, double *omega, double *Z0, double rtol, int32_t restart,
                                  int32_t maxit, int32_t precond, double *res_norm, int32_t *gmres_iters,
                                  double *gmres_relres) {
  if (!ctx || !omega || !Z0 || restart < 1 || restart > 500 || maxit < 1 || !(rtol > 0.0)) return FSE_E_INVAL;
  FSE_TRY(kr_alloc(ctx, restart));
  const Krylov k = kr_view(ctx, restart);
  double rn = 0.0;
  FSE_TRY(kr_evaluate(ctx, omega, Z0, k.r, &rn));
  if (res_norm) *res_norm = rn;
  // b = [-R; 0], held outside the GMRES work vectors
  const int N = k.N, nbk = (N + 255) / 256;
  double *b = k.b;
  hipLaunchKernelGGL(k_scale, dim3(nbk), dim3(256), 0, ctx->stream, N, -1.0, k.r, b);
  FSE_HIP(hipGetLastError());
  if (k.nu > 0) {
    FSE_HIP(hipMemsetAsync(b + N, 0, sizeof(double) * k.nu, ctx->stream));
    hipLaunchKernelGGL(k_kr_border, dim3((N * k.nu + 255) / 256), dim3(256), 0, ctx->stream, k.Bc, k.Pr, N, k.nu,
                       k.r, Z0, ctx->ktable_d, ctx->d - 1, ctx->e, 2.0 * M_PI / omega[0], ctx->U);
    FSE_HIP(hipGetLastError());
  }
  if (precond) FSE_TRY(kr_precond_build(k));
  int its = 0;
  double rel = 0.0;
  FSE_TRY(kr_gmres(k, b, precond != 0, rtol, restart, maxit, &its, &rel));
  if (gmres_iters) *gmres_iters = its;
  if (gmres_relres) *gmres_relres = rel;
  FSE_TRY(launch_axpby(ctx, N, 1.0, Z0, 1.0, k.x, Z0));
  if (k.nu > 0) {
    std::vector<double> dw(k.nu);
    FSE_HIP(hipMemcpyAsync(dw.data(), k.x + N, sizeof(double) * k.nu, hipMemcpyDeviceToHost, ctx->stream));
    FSE_HIP(hipStreamSynchronize(ctx->stream));
    for (int u = 0; u < k.nu; ++u) omega[ctx->e + u] += dw[u];
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  ctx->mf_ready = false;  // Z0 moved: the stored sensitivities belong to the old point
  return FSE_OK;
}

fse_status fse_newton_krylov_chord_step(fse_ctx *ctx, const double *omega, double *Z0, double rtol,
                                        int32_t restart, int32_t maxit, int32_t precond, double *res_norm,
                                        int32_t *gmres_iters, double *gmres_relres) {
  if (!ctx || !omega || !Z0 || restart < 1 || restart > 500 || maxit < 1 || !(rtol > 0.0)) return FSE_E_INVAL;
  if (ctx->d != ctx->e) {
    ctx->err = "chord steps need every base frequency known (d = e)";
    return FSE_E_UNSUPPORTED;
  }
  if (!ctx->mf_stored) {
    ctx->err = "no stored sensitivities: call fse_shooting_residual_matfree or fse_newton_krylov_step first";
    return FSE_E_INVAL;
  }
  FSE_TRY(kr_alloc(ctx, restart));
  const Krylov k = kr_view(ctx, restart);
  // the residual at (omega, Z0) from the states alone; PhiQU and rot_mf are left as they are
  FSE_TRY(integrate_points(ctx, 1, omega, Z0, nullptr, nullptr));
  FSE_TRY(launch_dft_residual(ctx, 1, Z0, k.r));
  double rn = 0.0;
  FSE_TRY(launch_norms(ctx, 1, k.r, &rn));
  if (res_norm) *res_norm = rn;
  const int N = k.N, nbk = (N + 255) / 256;
  hipLaunchKernelGGL(k_scale, dim3(nbk), dim3(256), 0, ctx->stream, N, -1.0, k.r, k.b);
  FSE_HIP(hipGetLastError());
  if (precond && !ctx->pc_ready) FSE_TRY(kr_precond_build(k));
  int its = 0;
  double rel = 0.0;
  FSE_TRY(kr_gmres(k, k.b, precond != 0, rtol, restart, maxit, &its, &rel));
  if (gmres_iters) *gmres_iters = its;
  if (gmres_relres) *gmres_relres = rel;
  FSE_TRY(launch_axpby(ctx, N, 1.0, Z0, 1.0, k.x, Z0));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  ctx->mf_ready = false;
  return FSE_OK;
}

}  // extern "C"
