// Internal declarations of the FSE-Shooting HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fse.h"

// ----------------------------------------------------------------------------- errors
#define FSE_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ctx->err = std::string("HIP error ") + hipGetErrorString(e_) + " at " +       \
                 __FILE__ + ":" + std::to_string(__LINE__);                        \
      return FSE_E_DEVICE;                                                         \
    }                                                                              \
  } while (0)

#define FSE_TRY(expr)                  \
  do {                                 \
    fse_status s_ = (expr);            \
    if (s_ != FSE_OK) return s_;       \
  } while (0)

// Device status word bits written by kernels (host reads after the stream syncs).
enum : int {
  DEV_OK = 0,
  DEV_NOCONV = 1,      // per-step Newton exceeded maxit
  DEV_SINGULAR = 2,    // zero or non-finite pivot
  DEV_NAN = 4,         // non-finite state
};

struct DevStatus {
  int flags;           // OR of DEV_* bits
  int first_step;      // smallest step index that raised DEV_NOCONV (or INT_MAX)
  int max_iters;       // largest per-step Newton iteration count
  int pad;
  unsigned long long total_iters;
};

// Per-call problem parameters passed to the trajectory kernels by value.
// Newmark step coefficients (h = 2 pi / S1; beta, gamma of the rule, 1/4 and 1/2 in App. E):
// a_{k+1} = c0 (q_{k+1} - q_k) - c1 u_k - c3 a_k,  u_{k+1} = c2 (q_{k+1} - q_k) - d1 u_k - d2 a_k,
// c0 = 1/(beta h^2), c1 = 1/(beta h), c2 = gamma/(beta h), c3 = 1/(2 beta) - 1,
// d1 = gamma/beta - 1, d2 = h (gamma/(2 beta) - 1); the step matrix is w1^2 c0 M + w1 c2 D + K
// and its right-hand side e + w1^2 M (c0 q + c1 u + c3 a) + w1 D (c2 q + d1 u + d2 a).
struct TrajParams {
  int n, bw, S1, e, d, St, W;   // sizes; W = B * St trajectories
  int maxit;
  double tol;
  double h, c0, c1, c2, c3, d1, d2;
  double phib;  // phase of forcing 1 at the start, per point index b (multiple shooting segments)
};

struct fse_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // sizes
  int n = 0, e = 0, d = 0, S1 = 0, U = 0, L = 0, St = 0, bw = 0;
  int Bmax = 1, prec = 0, maxit = 30;
  double tol = 1e-12;
  double nm_beta = 0.25, nm_gamma = 0.5;  // Newmark rule
  int seg_steps = 0;                      // > 0: integrate that many steps (multiple shooting)
  double seg_phase = 0.0;                 // forcing-1 phase at the start = seg_phase * point index
  int Wmax = 0;
  int nnz2 = 0, nnz3 = 0;

  // host tables
  std::vector<int32_t> ktable;      // [(L+1)][d-1]
  std::vector<int32_t> sidx;        // [d-1][St]
  std::vector<int32_t> Sdim;        // [d-1]
  std::vector<double> G, Gi;        // [St][U], [U][St]

  // device: system (banded full rows [n][2bw+1])
  double *Mb = nullptr, *Db = nullptr, *Kb = nullptr;
  double *F = nullptr;              // [e][n]
  // f_nl by output row: CSR over t2 (j,k,v) and t3 (j,k,l,v)
  int32_t *f2_ptr = nullptr, *f2_jk = nullptr;  double *f2_v = nullptr;
  int32_t *f3_ptr = nullptr, *f3_jkl = nullptr; double *f3_v = nullptr;
  // tangent lower band: contributions per entry p = m*(bw+1) + (i-m)
  int32_t *kt_ptr = nullptr, *kt_idx = nullptr;  double *kt_c = nullptr;  // idx pairs (p, r or -1)
  // velocity-dependent forces (factor indices n..2n-1 name qdot): C_t = d f / d qdot lists,
  // same layout as kt_*, and the velocity history [S1+1][n][Wmax] for the sensitivity pass
  bool has_vel = false;
  int32_t *ct_ptr = nullptr, *ct_idx = nullptr;  double *ct_c = nullptr;
  // unilateral contacts, CSR by DOF: cn_v holds (direction, gap, stiffness) per contact
  int32_t ncon = 0;
  int32_t *cn_ptr = nullptr;
  double *cn_v = nullptr;
  double *uhist = nullptr;
  // torus
  double *G_d = nullptr, *Gi_d = nullptr;
  int32_t *sidx_d = nullptr, *Sdim_d = nullptr, *ktable_d = nullptr;

  // device work buffers (sized for Bmax points)
  double *omega_d = nullptr;        // [Bmax][d]
  double *qhist = nullptr;          // [S1+1][n][Wmax]
  double *u0 = nullptr;             // [n][Wmax]
  double *zTw = nullptr;            // [2n][Wmax]
  double *state_scr = nullptr;      // per trajectory scratch for large systems
  size_t state_scr_elems = 0;       // its size in doubles (grown, never shrunk)
  double *PhiA = nullptr;           // [Wmax][n][2n]
  double *PhiQU = nullptr;          // [Wmax][2n][2n] internal when caller passes none
  double *sens_scr = nullptr;       // per block factor + per column y
  size_t sens_scr_elems = 0;
  DevStatus *status_d = nullptr;
  double *rot_d = nullptr;          // [Bmax][L] rotation angles alpha_l
  double *work_R = nullptr;         // [Bmax][2n][U]
  double *work_b = nullptr;         // bordered right-hand side [2nU + d - e]
  double *Zwork = nullptr;          // [Bmax][2n][U]
  double *Jw = nullptr;             // dense Jacobian / LU workspace [2nU][2nU]
  std::vector<double> F_host;   // unit-amplitude load vectors [e][n]
  std::vector<double> amp;      // forcing amplitudes [e]
  int32_t *piv_d = nullptr;
  int piv_n = 0;
  float *lu32 = nullptr;            // FP32 factor + one FP32 vector (mixed-precision dense solve)
  size_t lu32_elems = 0;
  double *ir = nullptr;             // refinement vectors b, x, r
  size_t ir_elems = 0;
  int last_refine = 0;              // refinement steps of the last mixed dense solve (-1: FP64 used)
  void *lu_part = nullptr;          // partial sums of the dense substitutions
  size_t lu_part_bytes = 0;
  double *lu_scr = nullptr;
  double *norm_d = nullptr;         // [Bmax] squared residual norms
  double *jacP = nullptr;           // [S~][U][U] Jacobian right factor
  double *sens_gscr = nullptr;      // factor scratch when it does not fit in LDS
  size_t sens_gscr_elems = 0;
  size_t Jw_elems = 0;
  // omega_1 derivative (arclength continuation)
  bool want_qhist = false;          // the next integration writes the displacement history
  bool wsens_generic = false;       // omega_1 sensitivity by the generic replay kernel
  double *dzw = nullptr;            // [2n][Wmax] d zbar(2 pi) / d omega_1
  double *zeros_d = nullptr;        // [Bmax][2n][U] zeros
  double *arc = nullptr;            // arclength vectors, 6 x (2nU + d - e + 1)
  size_t arc_elems = 0;
  double *wfac = nullptr;           // factors of T(q_{k+1}) for every step and trajectory
  size_t wfac_elems = 0;
  // matrix-free Newton-Krylov (k_krylov.hip)
  bool mf_ready = false;            // PhiQU holds the sensitivities of the evaluation at the current Z0
  bool mf_stored = false;           // PhiQU and rot_mf hold those of some earlier evaluation (chord steps)
  bool pc_ready = false;            // the preconditioner blocks in kr belong to the stored sensitivities
  double *rot_mf = nullptr;         // [L] rotation angles of the stored evaluation
  double *kr = nullptr;             // Krylov basis, work vectors, preconditioner blocks
  size_t kr_elems = 0;
  int32_t *kr_piv = nullptr;        // pivots of the preconditioner blocks
  // hyper-time FSE-Shooting (k_hypertime.hip)
  bool samples_in = false;          // the next integration starts from samples, not coefficients
  double *ht = nullptr;             // Gamma R Gamma^-1 per point, R Gamma^-1, residual
  size_t ht_elems = 0;
  // multiple FSE-Shooting (k_multiple.hip)
  double *mult = nullptr;           // next sections, residual [2][M][2n][U]
  size_t mult_elems = 0;

  // packed tensors for LDS staging: t2 (j | k << 16), t3 (j | k << 16, l)
  uint32_t *f2_pk = nullptr, *f3_pk = nullptr;
  // fused trajectory kernel: padded per-point bands [Bmax][n][2BW+1]
  double *Sp = nullptr, *Mwp = nullptr, *Dwp = nullptr, *Kp = nullptr;
  size_t fused_band_elems = 0;
  bool use_fused = true;

  // wide-band trajectory path (k_wide.hip): half bandwidths above the fused kernel's, lumped mass
  struct WideState *wide = nullptr;
  bool wide_forced = false;         // FSE_KERNELS=wide: take the wide path wherever it applies
  bool use_wide = true;             // FSE_KERNELS=generic turns it off

  // tuning
  int sens_cols = 64;               // columns per sensitivity work-group (generic kernel)
  int fused_ncw = 2;                // column waves per fused work-group
  bool ncw_autotune = true;         // tune fused_ncw on the first launch with sensitivities
  float ncw_ms[2] = {0.0f, 0.0f};   // autotuner timings for 1 and 2 column waves

  // timing of the last integration
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double last_ms[4] = {0, 0, 0, 0};
  int last_sens_launches = 0;
  int last_path = 0;                // trajectory kernels of the last integration: 0 generic, 1 fused, 2 wide
  int last_max_iters = 0;
  unsigned long long last_total_iters = 0;
};

// ----------------------------------------------------------------------------- host helpers (fse_api.hip)
// integrate B points (state, and sensitivities into Phi when non-null) with timing and status
fse_status integrate_points(fse_ctx *ctx, int B, const double *omega, const double *Z0, double *zT, double *Phi);
// the internal sensitivity buffer PhiQU [Wmax][2n][2n]
fse_status ensure_phi_buffer(fse_ctx *ctx);
// the dense Newton workspace Jw, at least Nb x Nb
fse_status ensure_dense_matrix(fse_ctx *ctx, size_t Nb);
// initial states of every trajectory straight from samples zbar(0) [B][2n][S~] (k_hypertime.hip)
fse_status launch_samples_in(fse_ctx *ctx, int B, const double *zbar0);

// ----------------------------------------------------------------------------- launches
// Trajectory integration (k_traj.hip)
fse_status reset_status(fse_ctx *ctx);
fse_status launch_idft(fse_ctx *ctx, int B, const double *Z0);
fse_status launch_state(fse_ctx *ctx, int B);
fse_status launch_sens(fse_ctx *ctx, int B, double *PhiQU);
fse_status launch_dft_residual(fse_ctx *ctx, int B, const double *Z0, double *R);
// (I (x) R(rho) Gamma^-1) zT - Z0 for terminal samples zT [2n][Wmax]
// rot: rotation angles [B][L] (device), or null for those of the last uploaded omega (rot_d)
fse_status launch_dft(fse_ctx *ctx, int B, const double *zT, const double *Z0, double *R,
                      const double *rot = nullptr);
fse_status launch_jacobian(fse_ctx *ctx, int B, const double *PhiQU, double *J, size_t ldJ);
fse_status launch_dRdw(fse_ctx *ctx, double *out, const double *R, const double *Z0, double omega1);
fse_status launch_border(fse_ctx *ctx, double *Jb, size_t ldJ, const double *R, const double *Z0,
                         double omega1);
fse_status launch_norms(fse_ctx *ctx, int B, const double *R, double *out_host);
fse_status launch_norm(fse_ctx *ctx, const double *x, size_t len, double *out_host);
fse_status launch_wsens(fse_ctx *ctx, int B, double *dzT);
fse_status launch_dRdp_rot(fse_ctx *ctx, int B, const double *omega, const double *R, const double *Z0,
                           double *dRdp);
fse_status launch_set_pcol(fse_ctx *ctx, double *A, size_t ldA, const double *col);
// Fused state + sensitivity kernel (k_fused.hip), half bandwidth <= 16
bool fused_supported(const fse_ctx *ctx);
// The fused kernel evaluates polynomial forces of q only; other systems take the generic kernels.
inline bool fused_eligible(const fse_ctx *ctx) {
  return ctx->use_fused && !ctx->has_vel && ctx->ncon == 0 && fused_supported(ctx);
}
void newmark_coefficients(const fse_ctx *ctx, TrajParams &p);  // h, c0 .. d2
fse_status launch_fused(fse_ctx *ctx, int B, double *Phi);
// compile-time half bandwidth (4, 6, 8, 12 or 16) the fused kernels use for this system
int fused_band_bucket(const fse_ctx *ctx);
// omega_1 sensitivity with the fused kernel's per-point bands (after a fused integration,
// k_wsens.hip); FSE_E_UNSUPPORTED when the generic replay must be used
fse_status launch_wsens_fused(fse_ctx *ctx, int B, double *dzT);
// Wide-band trajectory path (k_wide.hip): batched shared-S chord iteration for the states,
// per-trajectory banded LDL^T and MFMA block sweeps for the sensitivities.  wide_prepare is
// called by fse_init_torus with the full-row bands [n][2bw+1] of M, D, K, the f_nl rows (CSR by
// output index) and the tangent contribution lists (host); it keeps nothing when the system
// does not qualify (mass not diagonal, half bandwidth above 96, velocity-dependent forces, or
// staged rows beyond LDS).
fse_status wide_prepare(fse_ctx *ctx, const std::vector<double> &Mb, const std::vector<double> &Db,
                        const std::vector<double> &Kb, const std::vector<int32_t> &p2,
                        const std::vector<int32_t> &jk, const std::vector<int32_t> &p3,
                        const std::vector<int32_t> &jkl, const std::vector<int32_t> &ktp,
                        const std::vector<int32_t> &kti);
bool wide_eligible(const fse_ctx *ctx);
fse_status launch_wide_state(fse_ctx *ctx, int B);
fse_status launch_wide_sens(fse_ctx *ctx, int B, double *Phi);
void wide_free(fse_ctx *ctx);
// summed durations (HIP events on the context stream) and count of the sweep launches of the
// last wide-band integration with sensitivities (zero when there was none)
fse_status wide_sweep_timing(fse_ctx *ctx, double *ms_total, int *launches);
// Fixed scratch of the no-allocation J v (k_krylov.hip): 2^21 doubles (16 MiB) per GPU
constexpr size_t kNoAllocScratch = size_t(1) << 21;
constexpr int kMaxDevices = 64;
fse_status noalloc_setup(fse_ctx *ctx);   // once per device, from fse_init_torus
double *noalloc_scratch(int device);      // the device address taken by noalloc_setup, or null
// Dense linear algebra (k_linalg.hip)
fse_status dense_lu_solve(fse_ctx *ctx, double *A, int N, double *rhs);
// the two halves of dense_lu_solve: factor A (row-major N x N, in place, pivots piv[N]), then
// solve with the factor for one right-hand side (in place; enqueued, no synchronisation)
fse_status dense_lu_factor(fse_ctx *ctx, double *A, int N, int32_t *piv);
fse_status dense_lu_apply(fse_ctx *ctx, const double *A, int N, const int32_t *piv, double *rhs);
// FP32 LU of a copy of A with FP64 iterative refinement against A (kept) to 1e-10 of the
// right-hand side; FP64 LU if that fails
fse_status dense_lu_solve_refined(fse_ctx *ctx, double *A, int N, double *rhs);
// the dense solve of the Newton and arclength systems: refined in the mixed mode, FP64 otherwise
fse_status newton_dense_solve(fse_ctx *ctx, double *A, int N, double *rhs);
// `count` independent systems of one size: system z at A + z sA, pivots piv + z sp, rhs + z sx
fse_status dense_lu_apply_batched(fse_ctx *ctx, const double *A, size_t sA, int N, const int32_t *piv,
                                  size_t sp, double *rhs, size_t sx, int count);
fse_status launch_axpby(fse_ctx *ctx, int N, double a, const double *x, double b, const double *z, double *y);
fse_status launch_axpy(fse_ctx *ctx, int N, double alpha, const double *x, double *y);
fse_status launch_lincomb(fse_ctx *ctx, int N, const double *x, double alpha, const double *d, double *y);
fse_status lyapunov_qr(fse_ctx *ctx, const double *PhiQU, const double *omega_h, int N_Ly,
                       const double *Q0, double *sigma_h);
