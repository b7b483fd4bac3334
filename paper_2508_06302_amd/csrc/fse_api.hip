// C-ABI entry points of the FSE-Shooting library: context set-up on the host
// (torus tables of App. B / App. D, banded device storage of the system) and the
// orchestration of the device kernels for Sec. 3.3 steps 2-6 and App. F.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>

#include "fse_internal.h"

namespace {

// Harmonic table of App. B (Eqs. B1-B2).  d = 2: [k_2; 0].  d > 2 from K~^{d-1}:
// g-block rows [r, -k] for k in k_d (outer) and r in the nonzero rows (inner);
// b-block rows [r, k] for k in [k_d; 0] (outer) and r in all rows (inner).
std::vector<std::vector<int>> harmonic_table(const std::vector<std::vector<int>> &k) {
  std::vector<std::vector<int>> T;
  if (k.empty()) {
    T.push_back({});
    return T;
  }
  for (int v : k[0]) T.push_back({v});
  T.push_back({0});
  for (size_t j = 1; j < k.size(); ++j) {
    std::vector<std::vector<int>> nt;
    const size_t nz = T.size() - 1;
    for (int kd : k[j])
      for (size_t r = 0; r < nz; ++r) {
        auto row = T[r];
        row.push_back(-kd);
        nt.push_back(row);
      }
    std::vector<int> kd0 = k[j];
    kd0.push_back(0);
    for (int kv : kd0)
      for (size_t r = 0; r < T.size(); ++r) {
        auto row = T[r];
        row.push_back(kv);
        nt.push_back(row);
      }
    T.swap(nt);
  }
  return T;
}

struct Csr {
  const int32_t *ptr, *idx;
  const double *val;
};

fse_status csr_to_band(fse_ctx *ctx, const char *name, Csr a, int n, int bw,
                       std::vector<double> &band) {
  const int w = 2 * bw + 1;
  band.assign((size_t)n * w, 0.0);
  if (!a.ptr || !a.idx || !a.val) {
    ctx->err = std::string("matrix ") + name + ": null CSR array";
    return FSE_E_INVAL;
  }
  for (int i = 0; i < n; ++i) {
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      const int j = a.idx[p];
      if (j < 0 || j >= n || std::abs(j - i) > bw) {
        ctx->err = std::string("matrix ") + name + ": column index out of range";
        return FSE_E_INVAL;
      }
      band[(size_t)i * w + (j - i + bw)] += a.val[p];
    }
  }
  double mx = 0.0;
  for (double v : band) mx = std::max(mx, std::abs(v));
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < w; ++t) {
      const int j = i - bw + t;
      if (j < 0 || j >= n) continue;
      const double aij = band[(size_t)i * w + t];
      const double aji = band[(size_t)j * w + (i - j + bw)];
      if (std::abs(aij - aji) > 1e-12 * mx) {
        ctx->err = std::string("matrix ") + name + " is not symmetric";
        return FSE_E_INVAL;
      }
    }
  return FSE_OK;
}

int csr_halfband(Csr a, int n) {
  int b = 0;
  if (!a.ptr) return 0;
  for (int i = 0; i < n; ++i)
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) b = std::max(b, std::abs(a.idx[p] - i));
  return b;
}

template <typename T>
fse_status upload(fse_ctx *ctx, T **dst, const std::vector<T> &src) {
  const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
  if (hipMalloc((void **)dst, bytes) != hipSuccess) {
    ctx->err = "hipMalloc failed (" + std::to_string(bytes) + " bytes)";
    return FSE_E_NOMEM;
  }
  if (!src.empty()) FSE_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return FSE_OK;
}

fse_status alloc(fse_ctx *ctx, void **dst, size_t bytes) {
  if (hipMalloc(dst, std::max<size_t>(bytes, 8)) != hipSuccess) {
    ctx->err = "hipMalloc failed (" + std::to_string(bytes) + " bytes)";
    return FSE_E_NOMEM;
  }
  return FSE_OK;
}

fse_status init_impl(const fse_system *sys, const fse_torus_desc *desc, fse_ctx *ctx) {
  if (!sys || !desc) {
    ctx->err = "null system or torus descriptor";
    return FSE_E_INVAL;
  }
  const int n = sys->n;
  if (n <= 0 || sys->e < 1 || desc->d < 1 || desc->d > 4 || desc->e != sys->e || desc->e > desc->d ||
      desc->S1 < 1 || desc->max_batch < 1) {
    ctx->err = "invalid sizes: need n > 0, 1 <= e <= d <= 4, e == system e, S1 >= 1, max_batch >= 1";
    return FSE_E_INVAL;
  }
  if (desc->precision != FSE_PREC_FP64 && desc->precision != FSE_PREC_MIXED_FP32) {
    ctx->err = "unknown precision";
    return FSE_E_INVAL;
  }
  ctx->n = n;
  ctx->e = sys->e;
  ctx->d = desc->d;
  ctx->S1 = desc->S1;
  ctx->Bmax = desc->max_batch;
  ctx->prec = desc->precision;
  ctx->tol = desc->step_tol > 0 ? desc->step_tol : 1e-12;
  ctx->maxit = desc->step_maxit > 0 ? desc->step_maxit : 30;
  // FSE_KERNELS=fused|generic selects the trajectory kernels (tests cover both paths)
  // (fused where it applies, then the wide-band path, then generic; "wide" puts the wide-band
  // path first wherever it applies, "generic" turns both off)
  if (const char *kv = std::getenv("FSE_KERNELS")) {
    ctx->use_fused = std::strcmp(kv, "generic") != 0;
    ctx->use_wide = std::strcmp(kv, "generic") != 0;
    ctx->wide_forced = std::strcmp(kv, "wide") == 0;
  }
  // FSE_WSENS=generic keeps the omega_1 sensitivity on the generic replay kernel
  if (const char *kv = std::getenv("FSE_WSENS")) ctx->wsens_generic = std::strcmp(kv, "generic") == 0;
  if (const char *nc = std::getenv("FSE_FUSED_NCW")) {
    ctx->fused_ncw = std::max(1, std::atoi(nc));
    ctx->ncw_autotune = false;
  }
  FSE_HIP(hipGetDevice(&ctx->device));

  // ---- torus tables (App. B, App. D)
  std::vector<std::vector<int>> klists;
  int off = 0;
  for (int j = 0; j < ctx->d - 1; ++j) {
    const int Lj = desc->K_len ? desc->K_len[j] : 0;
    if (Lj < 1 || !desc->K_list || !desc->S) {
      ctx->err = "every torus direction needs at least one positive harmonic";
      return FSE_E_INVAL;
    }
    std::vector<int> kj(desc->K_list + off, desc->K_list + off + Lj);
    off += Lj;
    for (int a = 0; a < Lj; ++a)
      if (kj[a] <= 0 || (a > 0 && kj[a] <= kj[a - 1])) {
        ctx->err = "harmonic orders must be positive and strictly ascending";
        return FSE_E_INVAL;
      }
    const int Sj = desc->S[j];
    if (Sj < 2 * kj.back() + 1) {
      ctx->err = "Nyquist condition S_j >= 2 H_j + 1 violated (Sec. 3.1)";
      return FSE_E_INVAL;
    }
    klists.push_back(kj);
    ctx->Sdim.push_back(Sj);
  }
  auto T = harmonic_table(klists);
  ctx->L = (int)T.size() - 1;
  ctx->U = 2 * ctx->L + 1;
  const int dm1 = ctx->d - 1;
  ctx->ktable.assign((size_t)(ctx->L + 1) * std::max(dm1, 1), 0);
  for (int r = 0; r <= ctx->L; ++r)
    for (int j = 0; j < dm1; ++j) ctx->ktable[(size_t)r * dm1 + j] = T[r][j];
  int64_t St = 1;
  for (int s : ctx->Sdim) St *= s;
  ctx->St = (int)St;
  // sample coordinates, phi_2 fastest (Eq. D1)
  ctx->sidx.assign((size_t)std::max(dm1, 1) * St, 0);
  {
    int64_t inner = 1;
    for (int j = 0; j < dm1; ++j) {
      for (int64_t s = 0; s < St; ++s) ctx->sidx[(size_t)j * St + s] = (int)((s / inner) % ctx->Sdim[j]);
      inner *= ctx->Sdim[j];
    }
  }
  // Gamma / Gamma^-1 (Eqs. D2-D3) with angles reduced in integers over prod S_j
  ctx->G.assign((size_t)St * ctx->U, 0.0);
  ctx->Gi.assign((size_t)ctx->U * St, 0.0);
  const double twopi = 2.0 * M_PI;
  for (int64_t s = 0; s < St; ++s) {
    ctx->G[(size_t)s * ctx->U] = 1.0;
    ctx->Gi[(size_t)s] = 1.0 / (double)St;
    for (int l = 0; l < ctx->L; ++l) {
      int64_t num = 0;
      for (int j = 0; j < dm1; ++j) {
        const int64_t Sj = ctx->Sdim[j];
        int64_t m = ((int64_t)T[l][j] * ctx->sidx[(size_t)j * St + s]) % Sj;
        if (m < 0) m += Sj;
        num = (num + m * (St / Sj)) % St;
      }
      const double th = twopi * (double)num / (double)St;
      const double c = std::cos(th), sn = std::sin(th);
      ctx->G[(size_t)s * ctx->U + 2 * l + 1] = c;
      ctx->G[(size_t)s * ctx->U + 2 * l + 2] = sn;
      ctx->Gi[(size_t)(2 * l + 1) * St + s] = 2.0 * c / (double)St;
      ctx->Gi[(size_t)(2 * l + 2) * St + s] = 2.0 * sn / (double)St;
    }
  }

  // ---- system: band width from matrices and from the tensor index pairs
  Csr M{sys->M_ptr, sys->M_idx, sys->M_val}, D{sys->D_ptr, sys->D_idx, sys->D_val},
      K{sys->K_ptr, sys->K_idx, sys->K_val};
  int bw = std::max({csr_halfband(M, n), csr_halfband(D, n), csr_halfband(K, n)});
  if (sys->nnz2 < 0 || sys->nnz3 < 0 || (sys->nnz2 > 0 && (!sys->t2_idx || !sys->t2_val)) ||
      (sys->nnz3 > 0 && (!sys->t3_idx || !sys->t3_val)) || !sys->F) {
    ctx->err = "invalid tensor or load arrays";
    return FSE_E_INVAL;
  }
  // factor indices in [n, 2n) name qdot (velocity-dependent forces); the output index is a row
  bool vel = false;
  for (int64_t p = 0; p < sys->nnz2; ++p) {
    const int32_t *ix = sys->t2_idx + 3 * p;
    for (int a = 0; a < 3; ++a)
      if (ix[a] < 0 || ix[a] >= (a == 0 ? n : 2 * n)) {
        ctx->err = "t2 index out of range";
        return FSE_E_INVAL;
      }
    vel = vel || ix[1] >= n || ix[2] >= n;
    bw = std::max({bw, std::abs(ix[1] % n - ix[0]), std::abs(ix[2] % n - ix[0])});
  }
  for (int64_t p = 0; p < sys->nnz3; ++p) {
    const int32_t *ix = sys->t3_idx + 4 * p;
    for (int a = 0; a < 4; ++a)
      if (ix[a] < 0 || ix[a] >= (a == 0 ? n : 2 * n)) {
        ctx->err = "t3 index out of range";
        return FSE_E_INVAL;
      }
    vel = vel || ix[1] >= n || ix[2] >= n || ix[3] >= n;
    bw = std::max({bw, std::abs(ix[1] % n - ix[0]), std::abs(ix[2] % n - ix[0]), std::abs(ix[3] % n - ix[0])});
  }
  ctx->has_vel = vel;
  ctx->bw = bw;
  std::vector<double> Mb, Db, Kb;
  FSE_TRY(csr_to_band(ctx, "M", M, n, bw, Mb));
  FSE_TRY(csr_to_band(ctx, "D", D, n, bw, Db));
  FSE_TRY(csr_to_band(ctx, "K", K, n, bw, Kb));

  // f_nl rows (CSR by output index)
  ctx->nnz2 = (int)sys->nnz2;
  ctx->nnz3 = (int)sys->nnz3;
  std::vector<int32_t> p2(n + 1, 0), p3(n + 1, 0);
  for (int64_t p = 0; p < sys->nnz2; ++p) p2[sys->t2_idx[3 * p] + 1]++;
  for (int64_t p = 0; p < sys->nnz3; ++p) p3[sys->t3_idx[4 * p] + 1]++;
  for (int i = 0; i < n; ++i) {
    p2[i + 1] += p2[i];
    p3[i + 1] += p3[i];
  }
  std::vector<int32_t> jk((size_t)2 * sys->nnz2), jkl((size_t)3 * sys->nnz3);
  std::vector<double> v2(sys->nnz2), v3(sys->nnz3);
  {
    std::vector<int32_t> c2(p2.begin(), p2.end() - 1), c3(p3.begin(), p3.end() - 1);
    for (int64_t p = 0; p < sys->nnz2; ++p) {
      const int32_t *ix = sys->t2_idx + 3 * p;
      const int q = c2[ix[0]]++;
      jk[2 * q] = ix[1];
      jk[2 * q + 1] = ix[2];
      v2[q] = sys->t2_val[p];
    }
    for (int64_t p = 0; p < sys->nnz3; ++p) {
      const int32_t *ix = sys->t3_idx + 4 * p;
      const int q = c3[ix[0]]++;
      jkl[3 * q] = ix[1];
      jkl[3 * q + 1] = ix[2];
      jkl[3 * q + 2] = ix[3];
      v3[q] = sys->t3_val[p];
    }
  }
  // tangent contributions to the lower band, position p = m*(bw+1) + (i-m): d f / d q into
  // con (K_t), d f / d qdot into conv (C_t); the other factors a, b index y = [q; qdot]
  const int bp = bw + 1;
  std::vector<std::vector<std::pair<double, std::pair<int, int>>>> con((size_t)n * bp), conv((size_t)n * bp);
  auto add = [&](int i, int m, double c, int a, int b) {
    auto &dst = m < n ? con : conv;
    const int mm = m % n;
    if (i >= mm) dst[(size_t)mm * bp + (i - mm)].push_back({c, {a, b}});
  };
  for (int64_t p = 0; p < sys->nnz2; ++p) {
    const int32_t *ix = sys->t2_idx + 3 * p;
    const double v = sys->t2_val[p];
    add(ix[0], ix[1], v, ix[2], -1);
    add(ix[0], ix[2], v, ix[1], -1);
  }
  for (int64_t p = 0; p < sys->nnz3; ++p) {
    const int32_t *ix = sys->t3_idx + 4 * p;
    const double v = sys->t3_val[p];
    add(ix[0], ix[1], v, ix[2], ix[3]);
    add(ix[0], ix[2], v, ix[1], ix[3]);
    add(ix[0], ix[3], v, ix[1], ix[2]);
  }
  std::vector<int32_t> ktp((size_t)n * bp + 1, 0), kti, ctp((size_t)n * bp + 1, 0), cti;
  std::vector<double> ktc, ctc;
  for (size_t q = 0; q < con.size(); ++q) {
    ktp[q + 1] = ktp[q] + (int32_t)con[q].size();
    for (auto &c : con[q]) {
      ktc.push_back(c.first);
      kti.push_back(c.second.first);
      kti.push_back(c.second.second);
    }
    ctp[q + 1] = ctp[q] + (int32_t)conv[q].size();
    for (auto &c : conv[q]) {
      ctc.push_back(c.first);
      cti.push_back(c.second.first);
      cti.push_back(c.second.second);
    }
  }
  // both tangents must be symmetric (banded LDL^T): check at a random state y = [q; qdot];
  // column keys m >= n are the C_t block
  if (sys->nnz2 + sys->nnz3 > 0) {
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    std::vector<double> q(2 * (size_t)n);
    for (auto &v : q) v = uni(rng);
    std::map<std::pair<int, int>, double> kt;
    for (int64_t p = 0; p < sys->nnz2; ++p) {
      const int32_t *ix = sys->t2_idx + 3 * p;
      const double v = sys->t2_val[p];
      kt[{ix[0], ix[1]}] += v * q[ix[2]];
      kt[{ix[0], ix[2]}] += v * q[ix[1]];
    }
    for (int64_t p = 0; p < sys->nnz3; ++p) {
      const int32_t *ix = sys->t3_idx + 4 * p;
      const double v = sys->t3_val[p];
      kt[{ix[0], ix[1]}] += v * q[ix[2]] * q[ix[3]];
      kt[{ix[0], ix[2]}] += v * q[ix[1]] * q[ix[3]];
      kt[{ix[0], ix[3]}] += v * q[ix[1]] * q[ix[2]];
    }
    double mx = 0.0;
    for (auto &kv : kt) mx = std::max(mx, std::abs(kv.second));
    for (auto &kv : kt) {
      const int i = kv.first.first, m = kv.first.second, blk = m >= n ? n : 0;
      auto it = kt.find({m - blk, i + blk});
      const double other = it == kt.end() ? 0.0 : it->second;
      if (std::abs(kv.second - other) > 1e-9 * mx) {
        ctx->err = "tangent of f_nl is not symmetric (d f / d q and d f / d qdot must both be symmetric)";
        return FSE_E_UNSUPPORTED;
      }
    }
  }

  FSE_TRY(wide_prepare(ctx, Mb, Db, Kb, p2, jk, p3, jkl, ktp, kti));

  // ---- uploads
  FSE_TRY(upload(ctx, &ctx->Mb, Mb));
  FSE_TRY(upload(ctx, &ctx->Db, Db));
  FSE_TRY(upload(ctx, &ctx->Kb, Kb));
  ctx->F_host.assign(sys->F, sys->F + (size_t)sys->e * n);
  ctx->amp.assign(sys->e, 1.0);
  FSE_TRY(upload(ctx, &ctx->F, ctx->F_host));
  FSE_TRY(upload(ctx, &ctx->f2_ptr, p2));
  FSE_TRY(upload(ctx, &ctx->f2_jk, jk));
  FSE_TRY(upload(ctx, &ctx->f2_v, v2));
  FSE_TRY(upload(ctx, &ctx->f3_ptr, p3));
  FSE_TRY(upload(ctx, &ctx->f3_jkl, jkl));
  FSE_TRY(upload(ctx, &ctx->f3_v, v3));
  if (n < 65536) {
    std::vector<uint32_t> pk2((size_t)sys->nnz2), pk3((size_t)2 * sys->nnz3);
    for (int64_t q = 0; q < sys->nnz2; ++q) pk2[q] = (uint32_t)jk[2 * q] | ((uint32_t)jk[2 * q + 1] << 16);
    for (int64_t q = 0; q < sys->nnz3; ++q) {
      pk3[2 * q] = (uint32_t)jkl[3 * q] | ((uint32_t)jkl[3 * q + 1] << 16);
      pk3[2 * q + 1] = (uint32_t)jkl[3 * q + 2];
    }
    FSE_TRY(upload(ctx, &ctx->f2_pk, pk2));
    FSE_TRY(upload(ctx, &ctx->f3_pk, pk3));
  }
  if (vel) {
    if (ctc.empty()) ctc.assign(1, 0.0), cti.assign(2, 0);
    FSE_TRY(upload(ctx, &ctx->ct_ptr, ctp));
    FSE_TRY(upload(ctx, &ctx->ct_idx, cti));
    FSE_TRY(upload(ctx, &ctx->ct_c, ctc));
  }
  FSE_TRY(upload(ctx, &ctx->kt_ptr, ktp));
  FSE_TRY(upload(ctx, &ctx->kt_idx, kti));
  FSE_TRY(upload(ctx, &ctx->kt_c, ktc));
  FSE_TRY(upload(ctx, &ctx->G_d, ctx->G));
  FSE_TRY(upload(ctx, &ctx->Gi_d, ctx->Gi));
  FSE_TRY(upload(ctx, &ctx->sidx_d, ctx->sidx));
  FSE_TRY(upload(ctx, &ctx->Sdim_d, ctx->Sdim.empty() ? std::vector<int32_t>{1} : ctx->Sdim));
  FSE_TRY(upload(ctx, &ctx->ktable_d, ctx->ktable));

  // ---- work buffers
  ctx->Wmax = ctx->Bmax * ctx->St;
  const size_t W = ctx->Wmax;
  FSE_TRY(alloc(ctx, (void **)&ctx->omega_d, sizeof(double) * ctx->Bmax * ctx->d));
  FSE_TRY(alloc(ctx, (void **)&ctx->qhist, sizeof(double) * (size_t)(ctx->S1 + 1) * n * W));
  if (ctx->has_vel) FSE_TRY(alloc(ctx, (void **)&ctx->uhist, sizeof(double) * (size_t)(ctx->S1 + 1) * n * W));
  FSE_TRY(alloc(ctx, (void **)&ctx->u0, sizeof(double) * (size_t)n * W));
  FSE_TRY(alloc(ctx, (void **)&ctx->zTw, sizeof(double) * (size_t)2 * n * W));
  FSE_TRY(alloc(ctx, (void **)&ctx->status_d, sizeof(DevStatus)));
  FSE_TRY(alloc(ctx, (void **)&ctx->rot_d, sizeof(double) * ctx->Bmax * std::max(ctx->L, 1)));
  FSE_TRY(alloc(ctx, (void **)&ctx->rot_mf, sizeof(double) * std::max(ctx->L, 1)));
  FSE_TRY(alloc(ctx, (void **)&ctx->work_R, sizeof(double) * ctx->Bmax * 2 * n * ctx->U));
  FSE_TRY(alloc(ctx, (void **)&ctx->Zwork, sizeof(double) * std::max(ctx->Bmax, 2) * 2 * n * ctx->U));
  FSE_TRY(alloc(ctx, (void **)&ctx->norm_d, sizeof(double) * ctx->Bmax));
  for (auto &e : ctx->ev) FSE_HIP(hipEventCreate(&e));
  return FSE_OK;
}

void free_all(fse_ctx *ctx) {
  wide_free(ctx);
  void *ptrs[] = {ctx->Mb, ctx->Db, ctx->Kb, ctx->F, ctx->f2_ptr, ctx->f2_jk, ctx->f2_v,
                  ctx->f3_ptr, ctx->f3_jkl, ctx->f3_v, ctx->kt_ptr, ctx->kt_idx, ctx->kt_c,
                  ctx->G_d, ctx->Gi_d, ctx->sidx_d, ctx->Sdim_d, ctx->ktable_d, ctx->omega_d,
                  ctx->qhist, ctx->u0, ctx->zTw, ctx->state_scr, ctx->PhiA, ctx->PhiQU,
                  ctx->sens_scr, ctx->status_d, ctx->rot_d, ctx->rot_mf, ctx->work_R, ctx->Zwork, ctx->Jw,
                  ctx->piv_d, ctx->lu_scr, ctx->lu32, ctx->ir, ctx->lu_part, ctx->norm_d, ctx->jacP, ctx->sens_gscr,
                  ctx->Sp, ctx->Mwp, ctx->Dwp, ctx->Kp, ctx->work_b, ctx->dzw, ctx->zeros_d, ctx->arc, ctx->wfac, ctx->kr, ctx->kr_piv, ctx->ht, ctx->mult,
                  ctx->ct_ptr, ctx->ct_idx, ctx->ct_c, ctx->uhist, ctx->cn_ptr, ctx->cn_v};
  if (ctx->f2_pk) (void)hipFree(ctx->f2_pk);
  if (ctx->f3_pk) (void)hipFree(ctx->f3_pk);
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
}

fse_status check_status(fse_ctx *ctx) {
  DevStatus st;
  FSE_HIP(hipMemcpyAsync(&st, ctx->status_d, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  ctx->last_max_iters = st.max_iters;
  ctx->last_total_iters = st.total_iters;
  if (st.flags & DEV_SINGULAR) {
    ctx->err = "zero or non-finite pivot in a banded factorisation";
    return FSE_E_SINGULAR;
  }
  if (st.flags & DEV_NOCONV) {
    ctx->err = "per-step Newton did not converge (first failing step " + std::to_string(st.first_step) + ")";
    return FSE_E_NOCONV;
  }
  if (st.flags & DEV_NAN) {
    ctx->err = "non-finite state during integration";
    return FSE_E_NAN;
  }
  return FSE_OK;
}

fse_status upload_omega(fse_ctx *ctx, int B, const double *omega) {
  if (!omega) {
    ctx->err = "omega is null";
    return FSE_E_INVAL;
  }
  for (int b = 0; b < B * ctx->d; ++b)
    if (!(omega[b] > 0.0) || !std::isfinite(omega[b])) {
      ctx->err = "omega must be finite and positive";
      return FSE_E_INVAL;
    }
  FSE_HIP(hipMemcpyAsync(ctx->omega_d, omega, sizeof(double) * B * ctx->d, hipMemcpyHostToDevice,
                         ctx->stream));
  // rotation angles alpha_l = 2 pi k~_l . rho (Eq. 14), rho_j = omega_j / omega_1
  std::vector<double> rot((size_t)B * std::max(ctx->L, 1), 0.0);
  const int dm1 = ctx->d - 1;
  for (int b = 0; b < B; ++b)
    for (int l = 0; l < ctx->L; ++l) {
      double a = 0.0;
      for (int j = 0; j < dm1; ++j)
        a += (double)ctx->ktable[(size_t)l * dm1 + j] * (omega[b * ctx->d + 1 + j] / omega[b * ctx->d]);
      rot[(size_t)b * std::max(ctx->L, 1) + l] = 2.0 * M_PI * a;
    }
  FSE_HIP(hipMemcpyAsync(ctx->rot_d, rot.data(), sizeof(double) * rot.size(), hipMemcpyHostToDevice,
                         ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status integrate_impl(fse_ctx *ctx, int B, const double *omega, const double *Z0, double *zT,
                          double *Phi) {
  if (B < 1 || B > ctx->Bmax || !Z0) {
    ctx->err = "B out of range [1, max_batch] or Z0 null";
    return FSE_E_INVAL;
  }
  FSE_TRY(upload_omega(ctx, B, omega));
  if (Phi && Phi == ctx->PhiQU) {
    // the sensitivities kept for the matrix-free Jacobian are about to be overwritten
    ctx->mf_ready = false;
    ctx->mf_stored = false;
    ctx->pc_ready = false;
  }
  FSE_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
  if (ctx->samples_in)
    FSE_TRY(launch_samples_in(ctx, B, Z0));  // Z0 holds the samples zbar(0) [B][2n][S~]
  else
    FSE_TRY(launch_idft(ctx, B, Z0));
  FSE_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
  const bool wide = wide_eligible(ctx);
  const bool fused = !wide && fused_eligible(ctx);
  if (!fused && !wide && Phi && ctx->prec == FSE_PREC_MIXED_FP32) {
    ctx->err = "FP32 sensitivities need the fused kernel (half bandwidth <= 16, LDS fit) or the wide-band "
               "path (lumped mass, half bandwidth <= 96, average acceleration, no contacts)";
    return FSE_E_UNSUPPORTED;
  }
  ctx->last_path = fused ? 1 : wide ? 2 : 0;
  if (fused) {
    FSE_TRY(launch_fused(ctx, B, Phi));
    FSE_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
  } else if (wide) {
    FSE_TRY(launch_wide_state(ctx, B));
    FSE_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
    if (Phi) FSE_TRY(launch_wide_sens(ctx, B, Phi));
  } else {
    FSE_TRY(launch_state(ctx, B));
    FSE_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
    if (Phi) FSE_TRY(launch_sens(ctx, B, Phi));
  }
  FSE_HIP(hipEventRecord(ctx->ev[3], ctx->stream));
  if (zT) {
    // zTw is [2n][Wmax]; caller layout [B][2n][S~]
    const int n2 = 2 * ctx->n;
    for (int b = 0; b < B; ++b)
      FSE_HIP(hipMemcpy2DAsync(zT + (size_t)b * n2 * ctx->St, sizeof(double) * ctx->St,
                               ctx->zTw + (size_t)b * ctx->St, sizeof(double) * ctx->Wmax,
                               sizeof(double) * ctx->St, n2, hipMemcpyDeviceToDevice, ctx->stream));
  }
  FSE_HIP(hipEventRecord(ctx->ev[4], ctx->stream));
  FSE_HIP(hipEventSynchronize(ctx->ev[4]));
  float t_all = 0, t_idft = 0, t_state = 0, t_sens = 0;
  FSE_HIP(hipEventElapsedTime(&t_all, ctx->ev[0], ctx->ev[4]));
  FSE_HIP(hipEventElapsedTime(&t_idft, ctx->ev[0], ctx->ev[1]));
  FSE_HIP(hipEventElapsedTime(&t_state, ctx->ev[1], ctx->ev[2]));
  FSE_HIP(hipEventElapsedTime(&t_sens, ctx->ev[2], ctx->ev[3]));
  ctx->last_ms[0] = t_all;
  ctx->last_ms[1] = t_state;
  ctx->last_ms[2] = t_sens;
  ctx->last_ms[3] = t_idft;
  return check_status(ctx);
}

fse_status ensure_phi(fse_ctx *ctx) {
  if (!ctx->PhiQU) {
    const size_t W = ctx->Wmax, n = ctx->n;
    FSE_TRY(alloc(ctx, (void **)&ctx->PhiQU, sizeof(double) * W * 4 * n * n));
  }
  return FSE_OK;
}

}  // namespace

fse_status integrate_points(fse_ctx *ctx, int B, const double *omega, const double *Z0, double *zT, double *Phi) {
  return integrate_impl(ctx, B, omega, Z0, zT, Phi);
}

fse_status ensure_phi_buffer(fse_ctx *ctx) { return ensure_phi(ctx); }

// ============================================================================= C-ABI
void newmark_coefficients(const fse_ctx *ctx, TrajParams &p) {
  const double b = ctx->nm_beta, g = ctx->nm_gamma, h = 2.0 * M_PI / ctx->S1;
  p.h = h;
  p.c0 = 1.0 / (b * h * h);
  p.c1 = 1.0 / (b * h);
  p.c2 = g / (b * h);
  p.c3 = 1.0 / (2.0 * b) - 1.0;
  p.d1 = g / b - 1.0;
  p.d2 = h * (g / (2.0 * b) - 1.0);
}

extern "C" {

fse_status fse_init_torus(const fse_system *sys, const fse_torus_desc *desc, fse_ctx **out) {
  if (!out) return FSE_E_INVAL;
  *out = nullptr;
  fse_ctx *ctx = new (std::nothrow) fse_ctx();
  if (!ctx) return FSE_E_NOMEM;
  fse_status s = init_impl(sys, desc, ctx);
  if (s == FSE_OK) s = noalloc_setup(ctx);
  if (s != FSE_OK) {
    // keep the context alive so that fse_last_error can report; caller destroys it
    *out = ctx;
    return s;
  }
  *out = ctx;
  return FSE_OK;
}

fse_status fse_get_layout(const fse_ctx *ctx, int32_t *U, int32_t *Stilde, int32_t *half_band,
                          int32_t *ktable) {
  if (!ctx) return FSE_E_INVAL;
  if (U) *U = ctx->U;
  if (Stilde) *Stilde = ctx->St;
  if (half_band) *half_band = ctx->bw;
  if (ktable && ctx->d > 1) std::memcpy(ktable, ctx->ktable.data(), sizeof(int32_t) * ctx->ktable.size());
  return FSE_OK;
}

fse_status fse_set_stream(fse_ctx *ctx, void *hip_stream) {
  if (!ctx) return FSE_E_INVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return FSE_OK;
}

fse_status fse_integrate_batch(fse_ctx *ctx, int32_t B, const double *omega, const double *Z0,
                               double *zT, double *Phi) {
  if (!ctx) return FSE_E_INVAL;
  return integrate_impl(ctx, B, omega, Z0, zT, Phi);
}

fse_status fse_step_stats(const fse_ctx *ctx, int32_t *max_iters, int64_t *total_iters) {
  if (!ctx) return FSE_E_INVAL;
  if (max_iters) *max_iters = ctx->last_max_iters;
  if (total_iters) *total_iters = (int64_t)ctx->last_total_iters;
  return FSE_OK;
}

fse_status fse_shooting_residual_jacobian(fse_ctx *ctx, int32_t B, const double *omega,
                                          const double *Z0, double *R, double *rnorm, double *J,
                                          double *dRdw) {
  if (!ctx) return FSE_E_INVAL;
  if (!R) {
    ctx->err = "R must not be null";
    return FSE_E_INVAL;
  }
  const int nu = ctx->d - ctx->e;
  if (dRdw && nu == 0) {
    ctx->err = "dR/domega is defined for the unknown base frequencies only (d > e)";
    return FSE_E_INVAL;
  }
  double *phi = nullptr;
  if (J) {
    FSE_TRY(ensure_phi(ctx));
    phi = ctx->PhiQU;
  }
  FSE_TRY(integrate_impl(ctx, B, omega, Z0, nullptr, phi));
  FSE_TRY(launch_dft_residual(ctx, B, Z0, R));
  if (rnorm) FSE_TRY(launch_norms(ctx, B, R, rnorm));
  const size_t N = (size_t)2 * ctx->n * ctx->U;
  if (J) FSE_TRY(launch_jacobian(ctx, B, phi, J, N));
  if (dRdw) {
    for (int b = 0; b < B; ++b) {
      FSE_TRY(launch_dRdw(ctx, dRdw + (size_t)b * N * nu, R + (size_t)b * N, Z0 + (size_t)b * N,
                          omega[(size_t)b * ctx->d]));
    }
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

namespace {

// Residual, Newton matrix and right-hand side at (omega, Z0) for one point.  d = e: the
// Jacobian of Eq. (22).  d > e: bordered by dR/d omega_u and the phase rows of Eq. (18),
// Nb = N + d - e, row-major in Jb; rhs = [R; 0].
fse_status newton_system(fse_ctx *ctx, const double *omega, const double *Z0, double *Jb, double *rhs,
                         double *rn) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  FSE_TRY(ensure_phi(ctx));
  FSE_TRY(integrate_impl(ctx, 1, omega, Z0, nullptr, ctx->PhiQU));
  FSE_TRY(launch_dft_residual(ctx, 1, Z0, rhs));
  FSE_TRY(launch_norms(ctx, 1, rhs, rn));
  FSE_TRY(launch_jacobian(ctx, 1, ctx->PhiQU, Jb, (size_t)N + nu));
  if (nu > 0) {
    FSE_TRY(launch_border(ctx, Jb, (size_t)N + nu, rhs, Z0, omega[0]));
    FSE_HIP(hipMemsetAsync(rhs + N, 0, sizeof(double) * nu, ctx->stream));
  }
  return FSE_OK;
}

fse_status ensure_dp_buffers(fse_ctx *ctx) {
  const size_t N = (size_t)2 * ctx->n * ctx->U;
  if (!ctx->dzw) FSE_TRY(alloc(ctx, (void **)&ctx->dzw, sizeof(double) * 2 * ctx->n * ctx->Wmax));
  if (!ctx->zeros_d) {
    FSE_TRY(alloc(ctx, (void **)&ctx->zeros_d, sizeof(double) * ctx->Bmax * N));
    FSE_HIP(hipMemsetAsync(ctx->zeros_d, 0, sizeof(double) * ctx->Bmax * N, ctx->stream));
  }
  return FSE_OK;
}

// Integration of B points that also leaves the displacement history for the omega_1
// sensitivity (the fused kernel writes it only on request).
fse_status integrate_with_history(fse_ctx *ctx, int B, const double *omega, const double *Z0, double *Phi) {
  ctx->want_qhist = true;
  const fse_status st = integrate_impl(ctx, B, omega, Z0, nullptr, Phi);
  ctx->want_qhist = false;
  return st;
}

// dR/dp (p = omega_1 along the frequency conditions) after integrate_with_history and the
// residual R at the same points: the trajectory term through the DFT and rotation of
// d zbar(2 pi)/d omega_1, then, for d > e, minus rho_u dR/d omega_u.
fse_status dp_after_integration(fse_ctx *ctx, int B, const double *omega, const double *Z0, const double *R,
                                double *dRdp) {
  const int mi = ctx->last_max_iters;
  const unsigned long long ti = ctx->last_total_iters;
  FSE_TRY(reset_status(ctx));
  FSE_TRY(launch_wsens(ctx, B, ctx->dzw));
  const fse_status st = check_status(ctx);
  ctx->last_max_iters = mi;  // the step statistics stay those of the integration
  ctx->last_total_iters = ti;
  FSE_TRY(st);
  FSE_TRY(launch_dft(ctx, B, ctx->dzw, ctx->zeros_d, dRdp));
  FSE_TRY(launch_dRdp_rot(ctx, B, omega, R, Z0, dRdp));
  return FSE_OK;
}

// Square workspace for an Nb x Nb dense system (grown, never shrunk).
fse_status ensure_matrix(fse_ctx *ctx, size_t Nb) {
  if (ctx->Jw_elems < Nb * Nb) {
    if (ctx->Jw) (void)hipFree(ctx->Jw);
    ctx->Jw = nullptr;
    ctx->Jw_elems = 0;
    FSE_TRY(alloc(ctx, (void **)&ctx->Jw, sizeof(double) * Nb * Nb));
    ctx->Jw_elems = Nb * Nb;
  }
  return FSE_OK;
}

fse_status ensure_newton_buffers(fse_ctx *ctx) {
  const size_t N = (size_t)2 * ctx->n * ctx->U, Nb = N + (ctx->d - ctx->e);
  FSE_TRY(ensure_matrix(ctx, Nb));
  if (!ctx->work_b) FSE_TRY(alloc(ctx, (void **)&ctx->work_b, sizeof(double) * 2 * Nb));
  return FSE_OK;
}

}  // namespace

extern "C++" fse_status ensure_dense_matrix(fse_ctx *ctx, size_t Nb) { return ensure_matrix(ctx, Nb); }


fse_status fse_newton_step(fse_ctx *ctx, double *omega, double *Z0, double *res_norm) {
  if (!ctx || !Z0 || !omega) return FSE_E_INVAL;
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e, Nb = N + nu;
  FSE_TRY(ensure_newton_buffers(ctx));
  double rn = 0.0;
  double *rhs = ctx->work_b;
  FSE_TRY(newton_system(ctx, omega, Z0, ctx->Jw, rhs, &rn));
  if (res_norm) *res_norm = rn;
  // [J dRu; P 0] x = [R; 0], then Z0 -= x_Z, omega_u -= x_omega
  FSE_TRY(newton_dense_solve(ctx, ctx->Jw, Nb, rhs));
  FSE_TRY(launch_axpy(ctx, N, -1.0, rhs, Z0));
  if (nu > 0) {
    std::vector<double> xw(nu);
    FSE_HIP(hipMemcpyAsync(xw.data(), rhs + N, sizeof(double) * nu, hipMemcpyDeviceToHost, ctx->stream));
    FSE_HIP(hipStreamSynchronize(ctx->stream));
    for (int u = 0; u < nu; ++u) omega[ctx->e + u] -= xw[u];
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_newton_solve(fse_ctx *ctx, double *omega, double *Z0, double tol, int32_t maxit,
                            int32_t *iters, double *res_norm) {
  if (!ctx || !Z0 || !omega) return FSE_E_INVAL;
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e, Nb = N + nu, d = ctx->d;
  FSE_TRY(ensure_newton_buffers(ctx));
  double *rhs = ctx->work_b, *rtrial = ctx->work_b + Nb;
  // residual and Newton matrix at Z0; every accepted trial point below is evaluated with its
  // matrix, so the next iteration starts from a valid pair without integrating again
  double rn = INFINITY;
  FSE_TRY(newton_system(ctx, omega, Z0, ctx->Jw, rhs, &rn));
  bool have_J = true;
  std::vector<double> om(omega, omega + d), omt(d), xw(nu);
  int it = 0;
  for (; it < maxit && !(rn < tol); ++it) {
    if (!have_J) {
      double r0 = 0.0;
      FSE_TRY(newton_system(ctx, om.data(), Z0, ctx->Jw, rhs, &r0));
    }
    // rhs <- (Newton matrix)^-1 [R; 0]; the Newton direction is its negative
    FSE_TRY(newton_dense_solve(ctx, ctx->Jw, Nb, rhs));
    have_J = false;
    if (nu > 0) {
      FSE_HIP(hipMemcpyAsync(xw.data(), rhs + N, sizeof(double) * nu, hipMemcpyDeviceToHost, ctx->stream));
      FSE_HIP(hipStreamSynchronize(ctx->stream));
    }
    // backtracking on ||R||: accept (Z, omega_u) - lambda x once the residual decreases
    double lam = 1.0;
    bool accepted = false;
    for (int ls = 0; ls < 8 && !accepted; ++ls, lam *= 0.5) {
      FSE_TRY(launch_lincomb(ctx, N, Z0, -lam, rhs, ctx->Zwork));
      omt = om;
      for (int u = 0; u < nu; ++u) omt[ctx->e + u] -= lam * xw[u];
      double rt = INFINITY;
      const fse_status st = newton_system(ctx, omt.data(), ctx->Zwork, ctx->Jw, rtrial, &rt);
      if (st != FSE_OK && st != FSE_E_NOCONV && st != FSE_E_NAN && st != FSE_E_SINGULAR) return st;
      if (st == FSE_OK && rt < (1.0 - 1e-4 * lam) * rn) {
        FSE_HIP(hipMemcpyAsync(Z0, ctx->Zwork, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
        FSE_HIP(hipMemcpyAsync(rhs, rtrial, sizeof(double) * Nb, hipMemcpyDeviceToDevice, ctx->stream));
        FSE_HIP(hipStreamSynchronize(ctx->stream));
        om = omt;
        rn = rt;
        accepted = true;
        have_J = true;
      }
    }
    if (!accepted) {
      for (int i = 0; i < d; ++i) omega[i] = om[i];
      if (iters) *iters = it;
      if (res_norm) *res_norm = rn;
      ctx->err = "Newton line search failed to reduce the residual";
      return FSE_E_NOCONV;
    }
  }
  for (int i = 0; i < d; ++i) omega[i] = om[i];
  if (iters) *iters = it;
  if (res_norm) *res_norm = rn;
  if (!(rn < tol)) {
    ctx->err = "Newton did not reach the residual tolerance";
    return FSE_E_NOCONV;
  }
  return FSE_OK;
}

fse_status fse_set_newmark(fse_ctx *ctx, double beta, double gamma) {
  if (!ctx) return FSE_E_INVAL;
  if (!(beta > 0.0) || !(gamma > 0.0) || !std::isfinite(beta) || !std::isfinite(gamma)) {
    ctx->err = "Newmark parameters must be finite with beta > 0 and gamma > 0";
    return FSE_E_INVAL;
  }
  ctx->nm_beta = beta;
  ctx->nm_gamma = gamma;
  return FSE_OK;
}

fse_status fse_set_contacts(fse_ctx *ctx, int32_t m, const int32_t *dof, const int32_t *dir,
                            const double *gap, const double *stiff) {
  if (!ctx) return FSE_E_INVAL;
  if (m < 0 || (m > 0 && (!dof || !dir || !gap || !stiff))) {
    ctx->err = "invalid contact arrays";
    return FSE_E_INVAL;
  }
  const int n = ctx->n;
  for (int c = 0; c < m; ++c)
    if (dof[c] < 0 || dof[c] >= n || (dir[c] != 1 && dir[c] != -1) || !std::isfinite(gap[c]) ||
        !std::isfinite(stiff[c]) || stiff[c] < 0.0) {
      ctx->err = "contact " + std::to_string(c) + ": dof out of range, direction not +-1, or gap / stiffness "
                 "not finite (stiffness must be >= 0)";
      return FSE_E_INVAL;
    }
  std::vector<int32_t> ptr(n + 1, 0);
  for (int c = 0; c < m; ++c) ptr[dof[c] + 1]++;
  for (int i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  std::vector<double> v(3 * (size_t)m);
  for (int c = 0; c < m; ++c) {
    const int p = fill[dof[c]]++;
    v[3 * p] = (double)dir[c];
    v[3 * p + 1] = gap[c];
    v[3 * p + 2] = stiff[c];
  }
  // earlier work on the stream may still read the old lists
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->cn_ptr) (void)hipFree(ctx->cn_ptr);
  if (ctx->cn_v) (void)hipFree(ctx->cn_v);
  ctx->cn_ptr = nullptr;
  ctx->cn_v = nullptr;
  ctx->ncon = 0;
  if (m == 0) return FSE_OK;
  FSE_TRY(upload(ctx, &ctx->cn_ptr, ptr));
  FSE_TRY(upload(ctx, &ctx->cn_v, v));
  ctx->ncon = m;
  return FSE_OK;
}

fse_status fse_set_forcing(fse_ctx *ctx, const double *amp) {
  if (!ctx || !amp) return FSE_E_INVAL;
  const int n = ctx->n, e = ctx->e;
  std::vector<double> Fs((size_t)e * n);
  for (int f = 0; f < e; ++f) {
    if (!std::isfinite(amp[f])) {
      ctx->err = "non-finite forcing amplitude";
      return FSE_E_INVAL;
    }
    ctx->amp[f] = amp[f];
    for (int i = 0; i < n; ++i) Fs[(size_t)f * n + i] = amp[f] * ctx->F_host[(size_t)f * n + i];
  }
  FSE_HIP(hipMemcpyAsync(ctx->F, Fs.data(), sizeof(double) * Fs.size(), hipMemcpyHostToDevice, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_secant_predict(fse_ctx *ctx, int32_t np, const double *p_prev, const double *p_cur,
                              const double *p_next, const double *Z_prev, const double *Z_cur,
                              double *Z_next) {
  if (!ctx || np < 1 || !p_prev || !p_cur || !p_next || !Z_prev || !Z_cur || !Z_next) return FSE_E_INVAL;
  double num = 0.0, den = 0.0;
  for (int i = 0; i < np; ++i) {
    const double dp = p_cur[i] - p_prev[i];
    num += (p_next[i] - p_cur[i]) * dp;
    den += dp * dp;
  }
  if (!(den > 0.0)) {
    ctx->err = "secant predictor needs two distinct parameter points";
    return FSE_E_INVAL;
  }
  const double tau = num / den;
  const int N = 2 * ctx->n * ctx->U;
  FSE_TRY(launch_axpby(ctx, N, 1.0 + tau, Z_cur, -tau, Z_prev, Z_next));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_continuation(fse_ctx *ctx, int32_t P, const double *params, const double *Z_init,
                            double tol, int32_t maxit, double *Z_out, int32_t *iters, double *rnorm) {
  if (!ctx || P < 1 || !params || !Z_init || !Z_out || !iters || !rnorm) return FSE_E_INVAL;
  if (ctx->d != ctx->e) {
    ctx->err = "natural-parameter continuation needs every base frequency known (d = e)";
    return FSE_E_UNSUPPORTED;
  }
  const int np = ctx->d + ctx->e;
  const size_t N = (size_t)2 * ctx->n * ctx->U;
  constexpr int kMaxBisect = 6;
  // the last two solved points (requested or inserted): parameters on the host, tori on the
  // device; the secant predictor uses them, so inserted points sharpen the prediction
  double *hist = nullptr;
  FSE_TRY(alloc(ctx, (void **)&hist, sizeof(double) * 2 * N));
  double *Za = hist, *Zb = hist + N;
  std::vector<double> pa(np), pb(np);
  int solved = 0;
  fse_status result = FSE_OK;
  for (int j = 0; j < P && result == FSE_OK; ++j) {
    const double *pj = params + (size_t)j * np;
    double *Zj = Z_out + j * N;
    // targets still to reach on the way to p_j (a stack: the back is solved next)
    std::vector<std::vector<double>> targets{std::vector<double>(pj, pj + np)};
    int bisections = 0, total_it = 0;
    double rn = 0.0;
    while (!targets.empty() && result == FSE_OK) {
      const std::vector<double> pt = targets.back();
      result = fse_set_forcing(ctx, pt.data() + ctx->d);
      if (result != FSE_OK) break;
      hipError_t e = hipSuccess;
      if (solved == 0)
        e = hipMemcpyAsync(Zj, Z_init, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream);
      else if (solved == 1)
        e = hipMemcpyAsync(Zj, Zb, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream);
      else
        result = fse_secant_predict(ctx, np, pa.data(), pb.data(), pt.data(), Za, Zb, Zj);
      if (e != hipSuccess) result = FSE_E_DEVICE;
      if (result != FSE_OK) break;
      int32_t it = 0;
      std::vector<double> om(pt.begin(), pt.begin() + ctx->d);
      const fse_status st = fse_newton_solve(ctx, om.data(), Zj, tol, maxit, &it, &rn);
      total_it += it;
      if (st == FSE_OK) {
        // accept: shift the history
        if (hipMemcpyAsync(Za, Zb, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(Zb, Zj, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
          result = FSE_E_DEVICE;
          break;
        }
        pa = pb;
        pb = pt;
        ++solved;
        targets.pop_back();
      } else if ((st == FSE_E_NOCONV || st == FSE_E_NAN || st == FSE_E_SINGULAR) && solved > 0 &&
                 bisections < kMaxBisect) {
        // step control: insert the midpoint between the last solved point and this target
        std::vector<double> mid(np);
        for (int k = 0; k < np; ++k) mid[k] = 0.5 * (pb[k] + pt[k]);
        targets.push_back(mid);
        ++bisections;
      } else {
        result = st;
      }
    }
    iters[j] = result == FSE_OK ? total_it : -1;
    rnorm[j] = rn;
  }
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(hist);
  return result;
}

fse_status fse_residual_dp(fse_ctx *ctx, int32_t B, const double *omega, const double *Z0, double *R,
                           double *dRdp) {
  if (!ctx || !omega || !Z0 || !R || !dRdp) return FSE_E_INVAL;
  FSE_TRY(ensure_dp_buffers(ctx));
  FSE_TRY(integrate_with_history(ctx, B, omega, Z0, nullptr));
  FSE_TRY(launch_dft_residual(ctx, B, Z0, R));
  FSE_TRY(dp_after_integration(ctx, B, omega, Z0, R, dRdp));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

}  // extern "C"

namespace {

constexpr int kArcHalvings = 6;

// Extended matrix of the arclength corrector at (omega, Z0) (Eqs. C1, C3): rows [R; phase rows;
// t^T], columns [Z(0) (N), omega_u (d - e), p = omega_1], row-major with ld = Na = N + d - e + 1;
// rhs = [R; 0; 0].  col receives dR/dp (N).
fse_status arclength_system(fse_ctx *ctx, const double *omega, const double *Z0, const double *t, double *A,
                            double *rhs, double *col, double *rn) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  const size_t Na = (size_t)N + nu + 1;
  FSE_TRY(ensure_phi(ctx));
  FSE_TRY(ensure_dp_buffers(ctx));
  FSE_TRY(integrate_with_history(ctx, 1, omega, Z0, ctx->PhiQU));
  FSE_TRY(launch_dft_residual(ctx, 1, Z0, rhs));
  FSE_TRY(launch_norms(ctx, 1, rhs, rn));
  FSE_TRY(launch_jacobian(ctx, 1, ctx->PhiQU, A, Na));
  if (nu > 0) FSE_TRY(launch_border(ctx, A, Na, rhs, Z0, omega[0]));
  FSE_TRY(dp_after_integration(ctx, 1, omega, Z0, rhs, col));
  FSE_TRY(launch_set_pcol(ctx, A, Na, col));
  FSE_HIP(hipMemcpyAsync(A + (Na - 1) * Na, t, sizeof(double) * Na, hipMemcpyDeviceToDevice, ctx->stream));
  FSE_HIP(hipMemsetAsync(rhs + N, 0, sizeof(double) * (nu + 1), ctx->stream));
  return FSE_OK;
}

// Frequencies of the iterate X = [Z(0); omega_u; p]: omega_1 = p, the forcing frequencies at
// the ratios of omega_ref (frequency conditions), omega_u from X.
fse_status arc_frequencies(fse_ctx *ctx, const double *omega_ref, const double *X, std::vector<double> &om) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e, e = ctx->e;
  std::vector<double> tail(nu + 1);
  FSE_HIP(hipMemcpyAsync(tail.data(), X + N, sizeof(double) * (nu + 1), hipMemcpyDeviceToHost, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  const double p = tail[nu];
  om[0] = p;
  for (int j = 1; j < e; ++j) om[j] = omega_ref[j] / omega_ref[0] * p;
  for (int u = 0; u < nu; ++u) om[e + u] = tail[u];
  if (!(p > 0.0) || !std::isfinite(p)) {
    ctx->err = "arclength iterate left omega_1 > 0";
    return FSE_E_NAN;
  }
  return FSE_OK;
}

// Corrector of Eq. (C3): Newton on [F; t^T (X - X_pred)] from X = X_pred (in place).  On
// success A holds the extended matrix at the solution (last row t^T).
fse_status arc_corrector(fse_ctx *ctx, const double *omega_ref, double *X, const double *t, double tol,
                         int maxit, double *A, double *rhs, double *col, int *iters, double *rn,
                         std::vector<double> &om) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  const int Na = N + nu + 1;
  *rn = INFINITY;
  for (int k = 0;; ++k) {
    *iters = k;
    FSE_TRY(arc_frequencies(ctx, omega_ref, X, om));
    FSE_TRY(arclength_system(ctx, om.data(), X, t, A, rhs, col, rn));
    if (*rn < tol) return FSE_OK;
    if (k >= maxit || !std::isfinite(*rn)) {
      ctx->err = "arclength corrector did not reach the residual tolerance";
      return FSE_E_NOCONV;
    }
    FSE_TRY(newton_dense_solve(ctx, A, Na, rhs));
    FSE_TRY(launch_axpy(ctx, Na, -1.0, rhs, X));
  }
}

// Tangent of Eq. (C1) at the point where A was built: A y = e_last, t = y / ||y||_2.
fse_status arc_tangent(fse_ctx *ctx, double *A, double *y, double *t) {
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e;
  const int Na = N + nu + 1;
  const double one = 1.0;
  FSE_HIP(hipMemsetAsync(y, 0, sizeof(double) * Na, ctx->stream));
  FSE_HIP(hipMemcpyAsync(y + Na - 1, &one, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  FSE_TRY(newton_dense_solve(ctx, A, Na, y));
  double nrm = 0.0;
  FSE_TRY(launch_norm(ctx, y, (size_t)Na, &nrm));
  if (!(nrm > 0.0) || !std::isfinite(nrm)) {
    ctx->err = "degenerate tangent";
    return FSE_E_SINGULAR;
  }
  FSE_TRY(launch_axpby(ctx, Na, 1.0 / nrm, y, 0.0, y, t));
  return FSE_OK;
}

bool arc_retryable(fse_status st) {
  return st == FSE_E_NOCONV || st == FSE_E_NAN || st == FSE_E_SINGULAR;
}

}  // namespace

extern "C" {

fse_status fse_arclength(fse_ctx *ctx, int32_t P, const double *omega0, const double *Z_init, double ds,
                         double tol, int32_t maxit, double *Z_out, double *omega_out, double *steps,
                         int32_t *iters, double *rnorm) {
  if (!ctx || P < 1 || !omega0 || !Z_init || !Z_out || !omega_out || !steps || !iters || !rnorm || maxit < 0)
    return FSE_E_INVAL;
  if (!(ds != 0.0) || !std::isfinite(ds) || !(tol > 0.0)) {
    ctx->err = "arclength step must be finite and non-zero, tol positive";
    return FSE_E_INVAL;
  }
  const int N = 2 * ctx->n * ctx->U, nu = ctx->d - ctx->e, d = ctx->d, e = ctx->e;
  const size_t Na = (size_t)N + nu + 1;
  FSE_TRY(ensure_matrix(ctx, Na));
  if (ctx->arc_elems < 6 * Na) {
    if (ctx->arc) (void)hipFree(ctx->arc);
    ctx->arc = nullptr;
    ctx->arc_elems = 0;
    FSE_TRY(alloc(ctx, (void **)&ctx->arc, sizeof(double) * 6 * Na));
    ctx->arc_elems = 6 * Na;
  }
  double *X = ctx->arc, *Xj = X + Na, *t = Xj + Na, *rhs = t + Na, *y = rhs + Na, *col = y + Na;
  double *A = ctx->Jw;
  // X = [Z_init; omega_u; omega_1]; first tangent row sign(ds) e_p
  std::vector<double> tail(nu + 1);
  for (int u = 0; u < nu; ++u) tail[u] = omega0[e + u];
  tail[nu] = omega0[0];
  FSE_HIP(hipMemcpyAsync(X, Z_init, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
  FSE_HIP(hipMemcpyAsync(X + N, tail.data(), sizeof(double) * (nu + 1), hipMemcpyHostToDevice, ctx->stream));
  const double sgn = ds > 0.0 ? 1.0 : -1.0;
  FSE_HIP(hipMemsetAsync(t, 0, sizeof(double) * Na, ctx->stream));
  FSE_HIP(hipMemcpyAsync(t + Na - 1, &sgn, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<double> om(d);
  int it = 0;
  double rn = INFINITY;
  // point 0: corrected at fixed omega_1 (the row e_p^T dX = 0), then the tangent with e_p
  fse_status st = arc_corrector(ctx, omega0, X, t, tol, maxit, A, rhs, col, &it, &rn, om);
  if (st != FSE_OK) {
    iters[0] = -1;
    rnorm[0] = rn;
    return st;
  }
  const double s_max = std::fabs(ds);
  double s = s_max;
  for (int j = 0;; ++j) {
    FSE_HIP(hipMemcpyAsync(Z_out + (size_t)j * N, X, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream));
    for (int k = 0; k < d; ++k) omega_out[(size_t)j * d + k] = om[k];
    steps[j] = j == 0 ? 0.0 : s;
    iters[j] = it;
    rnorm[j] = rn;
    if (j + 1 == P) break;
    FSE_TRY(arc_tangent(ctx, A, y, t));
    FSE_HIP(hipMemcpyAsync(Xj, X, sizeof(double) * Na, hipMemcpyDeviceToDevice, ctx->stream));
    if (j > 0) s = std::min(2.0 * s, s_max);
    bool ok = false;
    for (int h = 0; h <= kArcHalvings; ++h) {
      FSE_TRY(launch_lincomb(ctx, (int)Na, Xj, s, t, X));  // predictor, Eq. (C2)
      st = arc_corrector(ctx, omega0, X, t, tol, maxit, A, rhs, col, &it, &rn, om);
      if (st == FSE_OK) {
        ok = true;
        break;
      }
      if (!arc_retryable(st)) return st;
      s *= 0.5;
    }
    if (!ok) {
      iters[j + 1] = -1;
      rnorm[j + 1] = rn;
      ctx->err = "arclength corrector failed after " + std::to_string(kArcHalvings) + " step halvings";
      return FSE_E_NOCONV;
    }
  }
  FSE_HIP(hipStreamSynchronize(ctx->stream));
  return FSE_OK;
}

fse_status fse_continuation_learned(fse_ctx *ctx, int32_t P, const double *params, const double *features,
                                    const double *Z_init, double tol, int32_t maxit, fse_learned *m,
                                    int32_t first_learned, double *Z_out, int32_t *iters, double *rnorm,
                                    int32_t *used) {
  if (!ctx || P < 1 || !params || !features || !Z_init || !Z_out || !iters || !rnorm || !used || !m)
    return FSE_E_INVAL;
  if (ctx->d != ctx->e) {
    ctx->err = "natural-parameter continuation needs every base frequency known (d = e)";
    return FSE_E_UNSUPPORTED;
  }
  const int np = ctx->d + ctx->e, nf = fse_learned_inputs(m);
  const size_t N = (size_t)2 * ctx->n * ctx->U;
  double *Zl = nullptr, *Rl = nullptr;
  FSE_TRY(alloc(ctx, (void **)&Zl, sizeof(double) * N));
  if (alloc(ctx, (void **)&Rl, sizeof(double) * N) != FSE_OK) {
    (void)hipFree(Zl);
    return FSE_E_NOMEM;
  }
  fse_status result = FSE_OK;
  for (int j = 0; j < P && result == FSE_OK; ++j) {
    const double *pj = params + (size_t)j * np;
    used[j] = 0;
    result = fse_set_forcing(ctx, pj + ctx->d);
    if (result != FSE_OK) break;
    double *Zj = Z_out + j * N;
    hipError_t e = hipSuccess;
    if (j == 0)
      e = hipMemcpyAsync(Zj, Z_init, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream);
    else if (j == 1)
      e = hipMemcpyAsync(Zj, Z_out, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream);
    else
      result = fse_secant_predict(ctx, np, pj - 2 * np, pj - np, pj, Zj - 2 * N, Zj - N, Zj);
    if (e != hipSuccess) result = FSE_E_DEVICE;
    if (result != FSE_OK) break;
    if (j >= first_learned) {
      // judge: the prediction with the smaller residual starts Newton
      double rs = INFINITY, rl = INFINITY;
      const fse_status s1 = fse_shooting_residual_jacobian(ctx, 1, pj, Zj, Rl, &rs, nullptr, nullptr);
      result = fse_learned_predict(m, features + (size_t)j * nf, Zl);
      if (result != FSE_OK) break;
      const fse_status s2 = fse_shooting_residual_jacobian(ctx, 1, pj, Zl, Rl, &rl, nullptr, nullptr);
      const bool ok1 = s1 == FSE_OK && std::isfinite(rs), ok2 = s2 == FSE_OK && std::isfinite(rl);
      if (ok2 && (!ok1 || rl < rs)) {
        if (hipMemcpyAsync(Zj, Zl, sizeof(double) * N, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
          result = FSE_E_DEVICE;
          break;
        }
        used[j] = 1;
      }
    }
    int32_t it = 0;
    double rn = 0.0;
    std::vector<double> om(pj, pj + ctx->d);
    const fse_status st = fse_newton_solve(ctx, om.data(), Zj, tol, maxit, &it, &rn);
    iters[j] = st == FSE_OK ? it : -1;
    rnorm[j] = rn;
    result = st;
  }
  (void)hipFree(Zl);
  (void)hipFree(Rl);
  return result;
}

fse_status fse_lyapunov(fse_ctx *ctx, const double *omega, const double *Z0, int32_t N_Ly,
                        const double *Q0, double *sigma) {
  if (!ctx || !Z0 || !sigma || N_Ly < 1) return FSE_E_INVAL;
  FSE_TRY(ensure_phi(ctx));
  FSE_TRY(integrate_impl(ctx, 1, omega, Z0, nullptr, ctx->PhiQU));
  return lyapunov_qr(ctx, ctx->PhiQU, omega, N_Ly, Q0, sigma);
}

fse_status fse_last_timing(const fse_ctx *ctx, double *ms4, int32_t *launches_out) {
  if (!ctx) return FSE_E_INVAL;
  if (ms4)
    for (int i = 0; i < 4; ++i) ms4[i] = ctx->last_ms[i];
  if (launches_out) *launches_out = ctx->last_sens_launches;
  return FSE_OK;
}

fse_status fse_last_kernel_timing(fse_ctx *ctx, int32_t *path, double *ms_total, int32_t *launches) {
  if (!ctx || !path || !ms_total || !launches) return FSE_E_INVAL;
  *path = ctx->last_path;
  *ms_total = 0.0;
  *launches = 0;
  if (ctx->last_path == 1) {
    // the fused kernel is one launch between the idft and end-of-integration events
    *ms_total = ctx->last_ms[1] + ctx->last_ms[2];
    *launches = 1;
  } else if (ctx->last_path == 2) {
    int l = 0;
    FSE_TRY(wide_sweep_timing(ctx, ms_total, &l));
    *launches = l;
  }
  return FSE_OK;
}

fse_status fse_get_tuning(const fse_ctx *ctx, int32_t *ncw, float *ms2) {
  if (!ctx) return FSE_E_INVAL;
  if (ncw) *ncw = ctx->fused_ncw;
  if (ms2) {
    ms2[0] = ctx->ncw_ms[0];
    ms2[1] = ctx->ncw_ms[1];
  }
  return FSE_OK;
}

const char *fse_last_error(const fse_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void fse_destroy(fse_ctx *ctx) {
  if (!ctx) return;
  free_all(ctx);
  delete ctx;
}

}  // extern "C"
