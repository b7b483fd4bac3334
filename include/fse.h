/*
 * fse.h -- C-ABI of the FSE-Shooting hot path on one MI355X (gfx950).
 *
 * FSE-Shooting (Fourier-series-expansion shooting, Wu, Hong, Li, Jiang 2025)
 * computes quasi-periodic responses of
 *
 *     M q'' + D q' + K q + f_nl(q) = sum_{i=1..e} F_i cos(omega_i t)       (Eq. 1, Eq. 25)
 *
 * by shooting on the Fourier coefficients Z(0) of the initial (d-1)-torus:
 * Z(0) -> z(0, phi~) (inverse DFT, Eq. 20) -> every trajectory integrated over
 * phi_1 in [0, 2 pi] by average-acceleration Newmark (App. E) -> z(2 pi, phi~)
 * -> Z(2 pi) (DFT, Eq. 21) -> R = (I (x) R(rho)) Z(2 pi) - Z(0) (Eqs. 15-16).
 *
 * Conventions (bit-exact parts of the contract):
 *   - harmonic table K~ of App. B (Eqs. B1-B2): (L+1) x (d-1) int32 rows, row-major,
 *     rows 0..L-1 the harmonic vectors k~_1..k~_L, last row zero;  U = 2L + 1;
 *   - Fourier coefficients Z: [2n][U], state-major (Eq. 10), state order [q; u]
 *     with u = dq/dphi_1 (App. E); column 0 the constant term, columns 2l-1 /
 *     2l the cos / sin coefficients of row l-1 of K~ (Eq. 11);
 *   - samples: S~ = prod S_j points, phi_2 fastest (Eq. D1); zbar: [2n][S~];
 *   - sensitivities Phi_s = d[q;u](2 pi) / d[q;u](0) (Eq. E8): [2n][2n] row-major.
 *
 * Memory: fse_init_torus reads HOST arrays and deep-copies them to the device.
 * Every array argument of the compute calls (omega excepted where noted) is a
 * DEVICE pointer (e.g. a torch tensor's data_ptr()) owned by the caller; work
 * is enqueued on the context stream (fse_set_stream) and the call returns after
 * that stream has completed it, unless stated otherwise.
 *
 * Errors: every call returns fse_status; FSE_OK == 0.  On error the message is
 * available from fse_last_error(ctx) and no output is guaranteed to be valid.
 * Calls on one context are not thread-safe; distinct contexts are independent.
 */
#ifndef FSE_H
#define FSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fse_ctx fse_ctx;

typedef enum {
  FSE_OK = 0,
  FSE_E_INVAL = 1,        /* bad argument: sizes, CSR structure, Nyquist, d > 4, e > d   */
  FSE_E_NOMEM = 2,        /* device allocation failed                                    */
  FSE_E_DEVICE = 3,       /* HIP runtime error                                           */
  FSE_E_NOCONV = 4,       /* per-step Newton did not converge (step index in message)    */
  FSE_E_SINGULAR = 5,     /* zero / non-finite pivot in a banded or dense factorisation  */
  FSE_E_NAN = 6,          /* non-finite state                                            */
  FSE_E_UNSUPPORTED = 7   /* valid request the library does not handle (message says why) */
} fse_status;

typedef enum {
  FSE_PREC_FP64 = 0,        /* FP64 everywhere                                            */
  FSE_PREC_MIXED_FP32 = 1   /* sensitivity state [Q; U; A] stored in FP32 (FP64 arithmetic),
                               Phi returned widened to FP64; state, residuals, Jacobian
                               assembly and Newton stay FP64.  The Newton iteration on the
                               FP64 residual refines away the Jacobian's FP32 error.
                               Needs the fused kernel (FSE_E_UNSUPPORTED otherwise). */
} fse_precision;

/* System of Eq. (1) with Theta = I.  Matrices in CSR (0-based, sorted column
 * indices, symmetric); f_nl(q)_i = sum t2 q_j q_k + sum t3 q_j q_k q_l with
 * index tuples (i,j,k) / (i,j,k,l) stored as rows of t2_idx / t3_idx.  The
 * tangent d f_nl / dq must be symmetric (forces derived from a potential,
 * as for the paper's von Karman and shell models); fse_init_torus checks it.
 * Velocity-dependent forces f_nl(q, qdot) (Eq. 1): a factor index j, k or l
 * in [n, 2n) names qdot_{index - n} (qdot = omega_1 dq/dphi_1); the output
 * index i stays in [0, n).  Then d f_nl / d qdot must be symmetric as well
 * (FSE_E_UNSUPPORTED otherwise), and such systems run on the generic trajectory
 * kernels (so the mixed-precision path returns FSE_E_UNSUPPORTED).
 * Indices outside these ranges return FSE_E_INVAL.
 * F: [e][n] load amplitude vectors, forcing i has frequency omega_i. */
typedef struct {
  int32_t n;
  const int32_t *M_ptr, *M_idx; const double *M_val;
  const int32_t *D_ptr, *D_idx; const double *D_val;
  const int32_t *K_ptr, *K_idx; const double *K_val;
  int64_t nnz2; const int32_t *t2_idx; const double *t2_val;
  int64_t nnz3; const int32_t *t3_idx; const double *t3_val;
  int32_t e; const double *F;
} fse_system;

/* Torus and time discretisation (Sec. 3.1, App. B, App. D, App. E).
 * K_len[j-2] = L_j and K_list the concatenated positive harmonic orders k_j
 * (ascending) for j = 2..d; S[j-2] = S_j >= 2 max(k_j) + 1 (Nyquist, Sec. 3.1);
 * S1 Newmark steps per 2 pi of phi_1 (beta = 1/4, gamma = 1/2).
 * step_tol / step_maxit: per-step Newton stops when ||dq||_inf <= step_tol *
 * ||q||_inf (or when the update stops shrinking below 1e3 step_tol, the FP64
 * noise floor); defaults 1e-12 / 30 when <= 0.  max_batch: continuation points
 * (omega vectors) a single call may integrate together. */
typedef struct {
  int32_t d, e;
  const int32_t *K_len;
  const int32_t *K_list;
  const int32_t *S;
  int32_t S1;
  double step_tol;
  int32_t step_maxit;
  int32_t max_batch;
  int32_t precision;      /* fse_precision */
} fse_torus_desc;

/* Builds the torus tables (harmonic table, grid, Gamma, Gamma^-1 of Eqs. D1-D3),
 * converts the system to banded device storage and allocates all work buffers
 * for up to max_batch points.  Host pointers.  *out receives the context. */
fse_status fse_init_torus(const fse_system *sys, const fse_torus_desc *desc, fse_ctx **out);

/* Layout queries (host outputs, any may be NULL): number of Fourier
 * coefficients U, number of samples S~, half bandwidth of the banded storage,
 * and the harmonic table [(U+1)/2][d-1] of App. B. */
fse_status fse_get_layout(const fse_ctx *ctx, int32_t *U, int32_t *Stilde,
                          int32_t *half_band, int32_t *ktable);

/* Stream (hipStream_t) on which all work of this context is enqueued; NULL is
 * the null stream.  The stream must belong to the context's device. */
fse_status fse_set_stream(fse_ctx *ctx, void *hip_stream);

/* Steps 2-3 of Sec. 3.3 for B <= max_batch points.  omega: HOST [B][d].
 * Z0: [B][2n][U].  zT (out): [B][2n][S~] terminal samples zbar(2 pi, phi~_s).
 * Phi (out, may be NULL): [B][S~][2n][2n] sensitivities (Eq. E8); computed only
 * when Phi != NULL.  Newton statistics of the state integration are available
 * through fse_step_stats. */
fse_status fse_integrate_batch(fse_ctx *ctx, int32_t B, const double *omega,
                               const double *Z0, double *zT, double *Phi);

/* Max and total per-step Newton iterations of the last integration (host). */
fse_status fse_step_stats(const fse_ctx *ctx, int32_t *max_iters, int64_t *total_iters);

/* Steps 2-5 of Sec. 3.3: residual R = (I (x) R(rho)) Z(2 pi) - Z(0) (Eq. 16),
 * [B][2n][U]; rnorm (HOST, may be NULL): ||R||_2 per point.
 * J (may be NULL): [B][2nU][2nU] row-major Jacobian of Eq. (22) (requires the
 * sensitivities).  dRdw (may be NULL, d > e only): [B][2nU][d-e] derivatives of R with
 * respect to the unknown base frequencies omega_{e+1..d} (Eqs. 23-24; the forcing does not
 * depend on them, so only the rotation term is present; d alpha_l / d omega_i is read as
 * 2 pi k_{i,l} / omega_1).  FSE_E_INVAL if dRdw is given with d = e. */
fse_status fse_shooting_residual_jacobian(fse_ctx *ctx, int32_t B, const double *omega,
                                          const double *Z0, double *R, double *rnorm,
                                          double *J, double *dRdw);

/* One Newton-Raphson update of step 6 of Sec. 3.3 for one point, dense LU with partial
 * pivoting in FP64.  d = e: every base frequency is a forcing frequency (the frequency
 * conditions of Eq. 17b hold exactly) and Z0 <- Z0 - J^-1 R.  d > e: the unknown base
 * frequencies omega_{e+1..d} join the unknowns and the system is bordered by dR/d omega_u
 * and the phase rows [(I (x) nabla_i) Z0]^T dZ = 0 of Eq. (18) (Sec. 3.2).
 * omega: HOST [d], in/out (entries e+1..d updated when d > e); Z0: [2n][U] in/out;
 * res_norm (HOST): ||R||_2 before the update. */
fse_status fse_newton_step(fse_ctx *ctx, double *omega, double *Z0, double *res_norm);

/* Newton iterations of fse_newton_step until ||R||_2 < tol (App. C stopping rule) or
 * maxit, with backtracking on ||R||_2 (a step is accepted once the residual decreases).
 * omega: HOST [d], in/out as in fse_newton_step; Z0 in/out.
 * iters / res_norm (HOST): iterations used and the final ||R||_2.
 * Returns FSE_E_NOCONV if the tolerance was not reached or no step reduced ||R||. */
fse_status fse_newton_solve(fse_ctx *ctx, double *omega, double *Z0, double tol,
                            int32_t maxit, int32_t *iters, double *res_norm);

/* Newmark rule of the trajectory integration (App. E uses the average acceleration,
 * beta = 1/4, gamma = 1/2, the default; other values are the general rule named in the
 * paper's outlook): q_{k+1} = q_k + h u_k + h^2 ((1/2 - beta) a_k + beta a_{k+1}),
 * u_{k+1} = u_k + h ((1 - gamma) a_k + gamma a_{k+1}).  Unconditionally stable for
 * 2 beta >= gamma >= 1/2; gamma > 1/2 damps numerically.  Applies to every later call
 * (states, sensitivities, d/d omega).  FSE_E_INVAL unless beta > 0 and gamma > 0, finite. */
fse_status fse_set_newmark(fse_ctx *ctx, double beta, double gamma);

/* Unilateral penalty contacts, a nonsmooth part of f_nl (the paper's conclusions recommend
 * the extension to nonsmooth systems without giving a form): contact c on DOF dof[c] with
 * direction dir[c] = +1 or -1, gap gap[c] and stiffness stiff[c] >= 0 adds
 * dir k max(dir q_i - gap, 0) to f_nl(q)_i.  The step Newton and the sensitivities use its
 * generalised derivative (k on the diagonal while dir q_i - gap > 0, nothing at or below
 * the gap), so Phi, J and dR/dp are the derivatives of the discrete map wherever no step
 * lands exactly on a gap.  Such systems run on the generic trajectory kernels, so the
 * mixed-precision path returns FSE_E_UNSUPPORTED.  All arrays HOST [m], copied; m = 0
 * removes the contacts.  Replaces the previous set; waits for the context's stream first.
 * Applies to every later call.  FSE_E_INVAL for a DOF outside [0, n), a direction other
 * than +-1, or a gap or stiffness that is not finite (or a negative stiffness). */
fse_status fse_set_contacts(fse_ctx *ctx, int32_t m, const int32_t *dof, const int32_t *dir,
                            const double *gap, const double *stiff);

/* Forcing amplitudes: the load vectors of Eq. (25) become amp_i F_i, with the F given
 * to fse_init_torus as amplitude 1 (the paper's examples list the amplitudes f_i in
 * Sec. 4, Tables 1-4).  amp: HOST [e].  Applies to every later call. */
fse_status fse_set_forcing(fse_ctx *ctx, const double *amp);

/* Secant predictor of a natural-parameter continuation (the zeroth-order form of the
 * predictor of App. C): Z_next = Z_cur + tau (Z_cur - Z_prev) with
 * tau = <p_next - p_cur, p_cur - p_prev> / ||p_cur - p_prev||^2.
 * p_prev, p_cur, p_next: HOST [np] parameter vectors; Z_*: [2n][U] (Z_next may alias
 * neither input).  FSE_E_INVAL if p_cur == p_prev. */
fse_status fse_secant_predict(fse_ctx *ctx, int32_t np, const double *p_prev, const double *p_cur,
                              const double *p_next, const double *Z_prev, const double *Z_cur,
                              double *Z_next);

/* Natural-parameter continuation over P points (App. C, secant predictor, step control).
 * params: HOST [P][d+e]; point j has omega = params[j][0:d] and forcing amplitudes
 * params[j][d:d+e].  Point 0 starts from Z_init [2n][U], point 1 from the solution of
 * point 0, every later point from the secant prediction of the two most recent solutions.
 * Each point is solved by fse_newton_solve(tol, maxit); when that fails, the parameter step
 * is halved by inserting the midpoint between the last solved point and the target (up to
 * 6 times per requested point; inserted points are solved but not returned).
 * Z_out: [P][2n][U] solutions; iters, rnorm: HOST [P] Newton iterations (including those
 * of inserted points) and final ||R||_2.  On failure at point j the status is returned with
 * iters[j] = -1 and later points are not touched.  The forcing amplitudes stay at those of
 * the last point attempted.  Needs d = e (FSE_E_UNSUPPORTED otherwise). */
fse_status fse_continuation(fse_ctx *ctx, int32_t P, const double *params, const double *Z_init,
                            double tol, int32_t maxit, double *Z_out, int32_t *iters,
                            double *rnorm);

/* dR/dp for the continuation parameter p = omega_1 (Sec. 3.2.1): the forcing frequencies
 * follow omega_1 at fixed ratios (frequency conditions omega_j = rho_j omega_1, j = 2..e) and
 * the unknown frequencies omega_{e+1..d} are held.  By Eqs. (23)-(24) this is
 * (I (x) R(rho) Gamma^-1) d zbar(2 pi)/d omega_1 - sum_u rho_u dR/d omega_u, where the
 * trajectory derivative is the exact derivative of the converged discrete Newmark map with
 * respect to the omega_1 of Eq. (E1) (App. E); the second sum is present for d > e only.
 * omega: HOST [B][d]; Z0: device [B][2n][U]; R, dRdp: device [B][2n][U] outputs (R as in
 * fse_shooting_residual_jacobian).  Errors as fse_integrate_batch. */
fse_status fse_residual_dp(fse_ctx *ctx, int32_t B, const double *omega, const double *Z0, double *R,
                           double *dRdp);

/* Pseudo-arclength continuation in omega_1 (App. C): tangent predictor of Eqs. (C1)-(C2)
 * and Newton corrections orthogonal to the tangent (Eq. C3) on the unknowns
 * X = [Z(0); omega_u; omega_1] of the continuation problem of Sec. 3.2.1 (phase rows of
 * Eq. 18 for d > e, forcing frequencies at the ratios of omega0).  The tangent has unit
 * 2-norm over X; the first one solves Eq. (C1) with the row e_p oriented by the sign of ds.
 * Point 0 is Z_init corrected at omega0 (fixed omega_1); every later point is predicted at
 * step s from the previous one and corrected until ||R||_2 < tol in at most maxit Newton
 * corrections.  Step control: a failed corrector is retried from the same point with s
 * halved (at most 6 times); after an accepted point s doubles back, never beyond |ds|.
 * omega0: HOST [d] (start; its ratios define the frequency conditions), Z_init: device
 * [2n][U].  Outputs: Z_out device [P][2n][U]; HOST omega_out [P][d], steps [P] (step taken,
 * 0 for point 0), iters [P] (corrections), rnorm [P] (final ||R||_2).  On failure at point
 * j the status is returned with iters[j] = -1; earlier points are valid.  One dense
 * (2nU + d - e + 1)^2 FP64 workspace is held by the context. */
fse_status fse_arclength(fse_ctx *ctx, int32_t P, const double *omega0, const double *Z_init, double ds,
                         double tol, int32_t maxit, double *Z_out, double *omega_out, double *steps,
                         int32_t *iters, double *rnorm);

/* ---------------------------------------------------------------- matrix-free Newton-Krylov
 * For unknown counts whose dense Jacobian is too large to factor, the Jacobian of Eq. (22) is
 * applied to vectors instead:
 *     J v = (I (x) R(rho) Gamma^-1) blkdiag_s(Phi_s) (I (x) Gamma) v - v,
 * using the trajectory sensitivities kept by the context (one point).  fse_jacobian_apply
 * applies J alone; fse_newton_krylov_step borders it for unknown frequencies (d > e). */

/* Residual R (device [2n][U], and ||R||_2 on the host if rnorm is non-null) at one point
 * (omega HOST [d], Z0 device [2n][U]); keeps the sensitivities of every trajectory in the
 * context for fse_jacobian_apply.  Errors as fse_integrate_batch. */
fse_status fse_shooting_residual_matfree(fse_ctx *ctx, const double *omega, const double *Z0, double *R,
                                         double *rnorm);

/* Jv = J v (device [2n][U] each, must not alias) with the sensitivities of the last
 * fse_shooting_residual_matfree; FSE_E_INVAL if there are none (or a Newton-Krylov step has
 * moved Z0 since). */
fse_status fse_jacobian_apply(fse_ctx *ctx, const double *v, double *Jv);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same product J v as fse_jacobian_apply, with the
 * same arguments (v, Jv: [2n][U] device arrays owned by the caller; the sensitivities are those
 * of the last fse_shooting_residual_matfree on this context), computed without any allocation.
 * Its intermediates (I (x) Gamma) v and Phi_s x_s use a fixed scratch of 2^21 doubles (16 MiB)
 * that the library holds on each GPU for the life of the process (its address is taken by
 * fse_init_torus); it serves 2 x 2n x (max_batch S~) <= 2^21, e.g. the 1872-DOF shell with 128
 * trajectories or the three-frequency beam with 1024.  Larger problems: FSE_E_UNSUPPORTED.  All
 * calls on one GPU share that scratch: calls that overlap on one GPU (two host threads, two
 * streams) race and must be serialised by the caller.  Enqueued on the context stream; returns
 * after the stream has completed it.  FSE_E_INVAL without sensitivities or on a null pointer. */
fse_status fse_jacobian_apply_noalloc(fse_ctx *ctx, const double *v, double *Jv);

/* One Newton update Z0 <- Z0 + dZ (Z0 device [2n][U], omega HOST [d]), with J dZ = -R solved
 * by restarted GMRES(restart) to ||J dZ + R|| <= rtol ||R|| or maxit iterations.  For d > e
 * the unknowns are [Z(0); omega_u] and the system is bordered as in fse_newton_step: the
 * columns dR/domega_u and the phase rows of Eq. (18) join the matrix-free J, GMRES runs on
 * 2nU + d - e unknowns, and omega[e..d-1] is updated in place (the preconditioner acts on the
 * Z(0) block only).  precond != 0 uses right preconditioning by
 * the harmonic-block matrix P = Phi_bar (x) R(rho) - I (Phi_bar the mean of the trajectory
 * sensitivities; P = J for a linear system).  Each of its blocks (one 2n x 2n, one 4n x 4n per
 * harmonic pair) is factored once per step.  HOST outputs (any may be NULL): res_norm =
 * ||R||_2 before the update, gmres_iters, gmres_relres = ||J dZ + R|| / ||R|| reached.
 * Device workspace: (restart + 8) vectors of 2nU + d - e doubles, 2 (d - e) border vectors of
 * 2nU doubles and the preconditioner blocks (2n)^2 (1 + 4 L) doubles, held by the context. */
fse_status fse_newton_krylov_step(fse_ctx *ctx, double *omega, double *Z0, double rtol, int32_t restart,
                                  int32_t maxit, int32_t precond, double *res_norm, int32_t *gmres_iters,
                                  double *gmres_relres);

/* Simplified (chord) Newton step for continuation sweeps, where the Jacobian changes little
 * from one point to the next: R at (omega HOST [d], Z0 device [2n][U]) from the states alone
 * (no sensitivities are propagated), then J dZ = -R by GMRES as in fse_newton_krylov_step but
 * with the stored J, that of the last fse_shooting_residual_matfree or fse_newton_krylov_step
 * evaluation on this context (its Phi_s and its rotation R(rho), possibly at another Z0, omega
 * or forcing), and Z0 <- Z0 + dZ.  The preconditioner blocks of the stored J are factored at
 * the first chord step after an evaluation and reused until the next one.  This is Newton's
 * method with a frozen Jacobian: it converges linearly, at a rate set by how far the stored J
 * is from the Jacobian at the current point.  d = e only (FSE_E_UNSUPPORTED otherwise);
 * FSE_E_INVAL without stored sensitivities (any call that writes the context's sensitivity
 * buffer, e.g. fse_shooting_residual_jacobian with J or fse_lyapunov, discards them).
 * Outputs and workspace as fse_newton_krylov_step. */
fse_status fse_newton_krylov_chord_step(fse_ctx *ctx, const double *omega, double *Z0, double rtol,
                                        int32_t restart, int32_t maxit, int32_t precond, double *res_norm,
                                        int32_t *gmres_iters, double *gmres_relres);

/* ---------------------------------------------------------------- hyper-time domain
 * FSE-Shooting with the sampled initial states as unknowns (Sec. 3.4, Eq. FSES_T):
 *     R(zbar(0), omega) = (I (x) Gamma R(rho) Gamma^-1) zbar(2 pi) - zbar(0),
 * zbar(0), zbar(2 pi) and R laid out [2n][S~] per point; unknowns (i, s) -> i S~ + s.
 * The paper gives this form no phase condition; with unknown frequencies (d > e) the Newton
 * step carries Eqs. (18) and (23)-(24) over through Z = Gamma^-1 zbar. */

/* omega HOST [B][d], zbar0 device [B][2n][S~]; outputs R device [B][2n][S~], rnorm HOST [B]
 * (may be NULL), J device [B][2nS~][2nS~] row-major or NULL (then no sensitivities are
 * propagated): J[(i, s), (j, t)] = (Gamma R Gamma^-1)[s, t] Phi_t[i, j] - delta.  Errors as
 * fse_integrate_batch. */
fse_status fse_hypertime_residual_jacobian(fse_ctx *ctx, int32_t B, const double *omega, const double *zbar0,
                                           double *R, double *rnorm, double *J);

/* One Newton update of the hyper-time unknowns (zbar0 device [2n][S~], in place) with a dense
 * LU of the (2nS~)^2 Jacobian held by the context; res_norm HOST = ||R||_2 before the update
 * (may be NULL).  For d > e the matrix is bordered by the columns
 * (I (x) Gamma dR(rho)/domega_u Gamma^-1) zbar(2 pi) and the phase rows
 * [(I (x) nabla_{phi_u}) Gamma^-1 zbar(0)]^T (I (x) Gamma^-1), and omega[e..d-1] (HOST, in/out)
 * is updated.  FSE_E_SINGULAR on a zero pivot. */
fse_status fse_hypertime_newton_step(fse_ctx *ctx, double *omega, double *zbar0, double *res_norm);

/* ---------------------------------------------------------------- multiple FSE-Shooting
 * The paper's first recommendation for future work (Sec. 5), in the classical multiple-
 * shooting form of Sec. 3: the period of phi_1 is cut into M segments of S1 / M steps and the
 * unknowns are the sections Z^(m) [2n][U~] of the torus at phi_1 = 2 pi m / M (basis of
 * Eq. 13 over the phases of the other frequencies at that moment).  Segment m starts on
 * section m with the forcing of frequency 1 at phase 2 pi m / M; with Eq. (16) per segment
 *     R_m = (I (x) R(rho / M)) Gamma^-1 zbar^(m)(2 pi / M) - Z^((m + 1) mod M).
 * M = 1 is FSE-Shooting.  1 <= M <= max_batch and S1 a multiple of M (FSE_E_INVAL
 * otherwise).  The segments run as one batch of M points. */

/* omega HOST [d], Zs device [M][2n][U~]; outputs R device [M][2n][U~], rnorm HOST (||R||_2
 * over all segments, may be NULL), J device [M 2nU~][M 2nU~] row-major or NULL: diagonal
 * block m the Eq. (22) operator of segment m without -I, block (m, m + 1 mod M) = -I, the
 * rest zero.  Errors as fse_integrate_batch. */
fse_status fse_multiple_residual_jacobian(fse_ctx *ctx, int32_t M, const double *omega, const double *Zs,
                                          double *R, double *rnorm, double *J);

/* One Newton update of all sections (Zs device [M][2n][U~], in place) with a dense LU of the
 * block-cyclic Jacobian held by the context; res_norm HOST = ||R||_2 before the update (may
 * be NULL).  For d > e the unknown frequencies join the unknowns as in fse_newton_step: the
 * matrix is bordered by dR_m/domega_u (through R(rho / M), d alpha / d omega_u =
 * 2 pi k_u / (M omega_1)) and by the phase rows of Eq. (18) on section 0, and omega[e..d-1]
 * (HOST, in/out) is updated.  FSE_E_SINGULAR on a zero pivot. */
fse_status fse_multiple_newton_step(fse_ctx *ctx, int32_t M, double *omega, double *Zs, double *res_norm);

/* ---------------------------------------------------------------- learned predictor
 * Initial iterates for new continuation parameters from the converged tori of earlier
 * points: a POD basis of the converged Z(0) (method of snapshots: Gram matrix in FP64,
 * cyclic Jacobi eigen-solver) and a multilayer perceptron p -> POD coefficients
 * (n_in -> hidden -> hidden -> rank, GELU(erf) hidden activations, FP32 weights, mean
 * squared error, AdamW), trained and evaluated by the library's own kernels.  This is an
 * addition to the paper's continuation (App. C), which predicts from previous solutions
 * only; the secant predictor stays the fallback (fse_continuation_learned).
 *
 * Parameter layout (FP32, one flat array of fse_learned_num_params values): for each
 * layer l = 1..3 its weight matrix W_l [out][in] row-major, then its bias [out]. */
typedef struct fse_learned fse_learned;

/* Creates a predictor for the unknowns of ctx (N = 2 n U per point) with n_in parameters,
 * `hidden` units per hidden layer and `rank` POD modes; uses ctx's stream.  ctx must
 * outlive the predictor.  Weights are zero until fse_learned_set_params. */
fse_status fse_learned_create(fse_ctx *ctx, int32_t n_in, int32_t hidden, int32_t rank,
                              fse_learned **out);
int64_t fse_learned_num_params(const fse_learned *m);
int32_t fse_learned_inputs(const fse_learned *m);   /* n_in, or -1 for NULL */
/* params: HOST FP32 [fse_learned_num_params]; copies in / out.  set_params also resets
 * the AdamW moments and step counter. */
fse_status fse_learned_set_params(fse_learned *m, const float *params);
fse_status fse_learned_get_params(const fse_learned *m, float *params);

/* POD of m_snap snapshots X [m_snap][N] (device, FP64, one converged Z(0) per row):
 * mean, then the leading `rank` modes of the centred snapshots.  sigma (HOST, may be NULL):
 * [min(m_snap, rank)] singular values of the centred snapshot matrix, descending.
 * 2 <= m_snap <= 128. */
fse_status fse_learned_fit_pod(fse_learned *m, int32_t m_snap, const double *X, double *sigma);
/* POD basis out: mean [N] and modes [N][rank] (device FP64, row-major). */
fse_status fse_learned_get_pod(const fse_learned *m, double *mean, double *modes);

/* Mean squared error and its gradients for a batch, without updating: x [B][n_in] and
 * t [B][rank] HOST FP32 (already normalised), grads HOST FP32 [num_params], loss HOST.
 * B <= 256.  Exposed so the hand-written backward pass can be checked. */
fse_status fse_learned_loss_grad(fse_learned *m, int32_t B, const float *x, const float *t,
                                 float *loss, float *grads);

/* `steps` full-batch AdamW steps on given normalised data: x [B][n_in], t [B][rank] HOST
 * FP32, B <= 256; loss_hist (HOST, may be NULL) [steps] loss before each step.  The step
 * counter and moments continue from earlier calls (fse_learned_set_params resets them). */
fse_status fse_learned_fit(fse_learned *m, int32_t B, const float *x, const float *t, int32_t steps,
                           double lr, double wd, double *loss_hist);

/* Trains on m_snap points: params P HOST [m_snap][n_in] (FP64), snapshots X device
 * [m_snap][N] (the ones given to fse_learned_fit_pod).  Inputs are standardised per component
 * with the training set's mean and deviation; the POD coefficients are centred and divided by
 * one common scale, the RMS deviation of the snapshots from their mean, so that the loss is the
 * mean squared error of Z(0) in the POD subspace (the modes are orthonormal); full-batch AdamW (lr,
 * beta 0.9 / 0.999, eps 1e-8, decoupled weight decay wd) for `epochs` steps.
 * loss_hist (HOST, may be NULL): [epochs] training loss in normalised units. */
fse_status fse_learned_train(fse_learned *m, int32_t m_snap, const double *P, const double *X,
                             int32_t epochs, double lr, double wd, double *loss_hist);

/* Prediction Z = mean + modes (sd_c * mlp((p - mu_p) / sd_p) + mu_c): p HOST [n_in],
 * Z device [N] (FP64). */
fse_status fse_learned_predict(fse_learned *m, const double *p, double *Z);
void fse_learned_destroy(fse_learned *m);

/* Raw network outputs for B <= 256 normalised inputs: x HOST [B][n_in], y HOST [B][rank]
 * (FP32).  bf16 != 0 runs the three layers as bfloat16 matrix-core products
 * (v_mfma_f32_16x16x16_bf16): weights and each layer's input rounded to bfloat16, nearest with
 * ties to even, products accumulated in FP32, bias and GELU in FP32.  bf16 = 0 is the FP32
 * network used in training. */
fse_status fse_learned_forward(fse_learned *m, int32_t B, const float *x, int32_t bf16, float *y);

/* Predictions for P <= 256 points at once (the batched form of fse_learned_predict):
 * params HOST [P][n_in], Z device [P][2n][U]; bf16 as in fse_learned_forward. */
fse_status fse_learned_predict_batch(fse_learned *m, int32_t P, const double *params, int32_t bf16, double *Z);

/* fse_continuation with a second predictor: from point first_learned on, the learned
 * prediction for features[j] (HOST [P][n_in], e.g. (omega_1, omega_2 / omega_1, f)) and the
 * secant prediction are both evaluated (one residual each) and Newton starts from the one
 * with the smaller ||R||_2, so the secant predictor is both the fallback and the judge.
 * used (HOST [P]): 1 where the learned prediction was taken, else 0.  Other arguments as
 * fse_continuation. */
fse_status fse_continuation_learned(fse_ctx *ctx, int32_t P, const double *params,
                                    const double *features, const double *Z_init, double tol,
                                    int32_t maxit, fse_learned *m, int32_t first_learned,
                                    double *Z_out, int32_t *iters, double *rnorm, int32_t *used);

/* Lyapunov exponents of App. F from the sensitivities at Z0: Psi_s of Eq. (F3),
 * trigonometric interpolation on the torus basis at phi~ = 2 pi (i-1) rho,
 * N_Ly steps of Gram-Schmidt as Householder QR with positive diagonal.
 * Q0: [2n][2n] initial orthonormal basis or NULL for the identity.
 * sigma (HOST out): [2n] exponents in QR column order (1/s). */
fse_status fse_lyapunov(fse_ctx *ctx, const double *omega, const double *Z0, int32_t N_Ly,
                        const double *Q0, double *sigma);

/* Device time (ms, HIP events on the context stream) of the kernels of the
 * last fse_integrate_batch: [0] total, [1] state integration, [2] sensitivity
 * propagation, [3] AFT; launches_out: launches of the sensitivity kernel. */
fse_status fse_last_timing(const fse_ctx *ctx, double *ms4, int32_t *launches_out);

/* Autotuner of the fused trajectory kernel: the first launch with sensitivities times each
 * candidate number of sensitivity-column waves per work-group (1 and 2) and keeps the
 * fastest.  ncw (HOST): the count in use; ms2 (HOST [2], may be NULL): the timed launches
 * (0 until tuned).  Setting FSE_FUSED_NCW in the environment before fse_init_torus fixes
 * the count and skips the tuning. */
/* Timing of the dominant trajectory kernel of the last integration, from HIP events recorded on
 * the context stream around its launches (host outputs): path 1 = the fused state + sensitivity
 * kernel (one launch), 2 = the wide-band sensitivity sweep k_wide_sweep (one launch per Newmark
 * step; the summed durations and the count), 0 = the generic kernels (ms_total 0).  Used to
 * relate algorithmic work to kernel time (App. E, Eqs. E8-E9).  FSE_E_INVAL on a null pointer. */
fse_status fse_last_kernel_timing(fse_ctx *ctx, int32_t *path, double *ms_total, int32_t *launches);

fse_status fse_get_tuning(const fse_ctx *ctx, int32_t *ncw, float *ms2);

const char *fse_last_error(const fse_ctx *ctx);
void fse_destroy(fse_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FSE_H */
