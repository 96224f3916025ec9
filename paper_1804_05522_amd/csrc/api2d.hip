// Host side of the 2D solver (C ABI fde2d_*): shift selection, the batched
// shifted operator, and the factored-ADI step with exact-residual corrections.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

namespace {

enum { kR_R0 = 0, kR_D0 = 1, kR_D1 = 2, kR_X0 = 3, kR_X1 = 4, kR_T = 5, kR_C = 6, kR_ZERO = 7, kR_E0 = 8, kR_E1 = 9,
       kR_CAP = 10,   // bit mask of the work slots whose recompression hit its rank cap above its tolerance
       kR_K0 = 11, kR_K1 = 12,   // rank of the correction sum X_corr (ping-pong)
       kR_Q1 = 13, kR_Q2 = 14,   // ranks of the orthonormalised sketches of a dense compression
       kR_EK1 = 15, kR_EK2 = 16, // extended Krylov: ranks of a new A-side block's two orthonormalisations,
       kR_EQ1 = 17, kR_EQ2 = 18, // of the projected solution's range,
       kR_EK3 = 19, kR_EK4 = 20, // and of a new B-side block's
       kR_N = 21 };
constexpr int kMaxCorrections = 6;   // correction sweeps of a step after the first
constexpr int kSketch = 32;          // sketch columns of a dense compression

// ---------- Zolotarev shifts for two real intervals (host, FP64) ----------
double ellip_K(double k) {           // complete elliptic integral of the first kind, modulus k (AGM)
  double a = 1.0, b = std::sqrt(1.0 - k * k);
  for (int it = 0; it < 80 && std::fabs(a - b) > 1e-16 * a; ++it) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

double ellip_dn(double u, double k) { // Jacobi dn(u | k) by the AGM / descending Landen scheme
  std::vector<double> a{1.0}, c{k};
  double b = std::sqrt(1.0 - k * k);
  while (std::fabs(c.back()) > 1e-16 && a.size() < 80) {
    const double an = 0.5 * (a.back() + b), cn = 0.5 * (a.back() - b);
    b = std::sqrt(a.back() * b);
    a.push_back(an);
    c.push_back(cn);
  }
  const int N = int(a.size()) - 1;
  double phi = std::ldexp(1.0, N) * a[N] * u, prev = phi;
  for (int n = N; n >= 1; --n) {
    prev = phi;
    phi = 0.5 * (phi + std::asin(c[n] * std::sin(phi) / a[n]));
  }
  return std::cos(phi) / std::cos(prev - phi);
}

// Optimal rational r(z) = prod (z - p_j)/(z + q_j) for |r| small on [a1,b1] (spectrum of A)
// and large on [-b2,-a2] (minus the spectrum of B): the symmetric problem on
// [-alpha,-1] U [1,alpha] has zeros alpha dn((2j-1)K/(2n), k'), k' = sqrt(1 - 1/alpha^2),
// mapped back by the Moebius transformation fixing the cross ratio.
void zolotarev_shifts(double a1, double b1, double a2, double b2, int n, std::vector<double>& p,
                      std::vector<double>& q) {
  const double gam = (a1 + b2) * (b1 + a2) / ((a1 + a2) * (b1 + b2));
  const double alp = 2.0 * gam - 1.0 + 2.0 * std::sqrt(std::max(gam * gam - gam, 0.0));
  const double kp = std::sqrt(std::max(1.0 - 1.0 / (alp * alp), 0.0));
  const double K = ellip_K(kp);
  auto T = [&](double z) {   // maps -1 -> -a2, 1 -> a1, alpha -> b1
    const double z1 = -1.0, z2 = 1.0, z3 = alp, w1 = -a2, w2 = a1, w3 = b1;
    const double R = (z - z1) * (z2 - z3) / ((z - z3) * (z2 - z1));
    const double S = R * (w2 - w1) / (w2 - w3);
    return (w1 - S * w3) / (1.0 - S);
  };
  p.resize(n);
  q.resize(n);
  for (int j = 0; j < n; ++j) {
    const double z = alp * ellip_dn((2.0 * j + 1.0) * K / (2.0 * n), kp);
    p[j] = T(z);
    q[j] = -T(-z);
  }
}

// max over [a1,b1] of |r| times max over [a2,b2] of |1/r(-mu)| on log grids
double zolotarev_bound(double a1, double b1, double a2, double b2, const std::vector<double>& p,
                       const std::vector<double>& q) {
  double e1 = 0.0, e2 = 0.0;
  const int S = 2000;
  for (int s = 0; s < S; ++s) {
    const double l = a1 * std::pow(b1 / a1, double(s) / (S - 1));
    const double m = a2 * std::pow(b2 / a2, double(s) / (S - 1));
    double r1 = 1.0, r2 = 1.0;
    for (size_t j = 0; j < p.size(); ++j) {
      r1 *= std::fabs((l - p[j]) / (l + q[j]));
      r2 *= std::fabs((m - q[j]) / (m + p[j]));
    }
    e1 = std::max(e1, r1);
    e2 = std::max(e2, r2);
  }
  return e1 * e2;
}

template <typename T>
hodlr_status plan_alloc(fde2d_plan p, T** ptr, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (p->sizing || p->ws) {
    const size_t off = (p->ws_used + 255) & ~size_t(255);
    if (!p->sizing && off + bytes > p->ws_bytes) return HODLR_EWORKSPACE;
    p->ws_used = off + bytes;
    *ptr = p->sizing ? nullptr : reinterpret_cast<T*>(p->ws + off);
    return HODLR_OK;
  }
  void* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) return HODLR_ENOMEM;
  p->allocs.push_back(q);
  *ptr = static_cast<T*>(q);
  return HODLR_OK;
}

Grp grp(const double* ptr, int64_t ld, const int32_t* cdev, int cnt, double s) { return Grp{ptr, ld, cdev, cnt, s}; }
Grp grp_none() { return Grp{nullptr, 0, nullptr, 0, 0.0}; }

// Unit lists of work slot `slot` for jobs of rows_x x rows_y factors (gram
// chunks of both sides, their two reductions, form chunks), uploaded only
// when the slot's row counts change.
hodlr_status ensure_units(fde2d_plan P, int slot, int64_t rows_x, int64_t rows_y, hipStream_t s) {
  if (P->unit_rows[slot][0] == rows_x && P->unit_rows[slot][1] == rows_y) return HODLR_OK;
  const int cx = int((rows_x + kLrRows - 1) / kLrRows), cy = int((rows_y + kLrRows - 1) / kLrRows);
  const int fx = int((rows_x + 255) / 256), fy = int((rows_y + 255) / 256);
  LrUnit* du = P->units + int64_t(slot) * P->slot_units;
  ReduceUnit* dr = reinterpret_cast<ReduceUnit*>(du + P->cap_gram);
  LrUnit* dfu = du + P->cap_gram + 2;
  std::vector<LrUnit> units, fu;
  std::vector<ReduceUnit> reds;
  int out = 0;
  for (int side = 0; side < 2; ++side) {
    const int chunks = side == 0 ? cx : cy;
    reds.push_back(ReduceUnit{out, chunks, 2 * slot + side, 0});
    for (int c = 0; c < chunks; ++c) units.push_back(LrUnit{slot, side, c, out++});
    for (int c = 0; c < (side == 0 ? fx : fy); ++c) fu.push_back(LrUnit{slot, side, c, 0});
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(du, units.data(), units.size() * sizeof(LrUnit), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dr, reds.data(), reds.size() * sizeof(ReduceUnit), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dfu, fu.data(), fu.size() * sizeof(LrUnit), hipMemcpyHostToDevice));
  P->unit_rows[slot][0] = rows_x;
  P->unit_rows[slot][1] = rows_y;
  return HODLR_OK;
}

// Enqueue one low-rank job on work slot `slot` (Gram, transfer-matrix and
// norm storage): Grams of both sides, then either the recompression (core +
// forms) or only the norm.  The descriptor is a kernel argument; the unit
// lists of a slot are uploaded when its row counts change, so a call copies
// nothing from the host.
hodlr_status run_lr(fde2d_plan P, const LrJob& job, int slot, bool recompress, hipStream_t s) {
  LrJob jb = job;
  jb.flops = P->counters;
  jb.gx = 2 * slot;
  jb.gy = 2 * slot + 1;
  jb.mslot = slot;
  const int cx = int((jb.rows_x + kLrRows - 1) / kLrRows), cy = int((jb.rows_y + kLrRows - 1) / kLrRows);
  const int fx = int((jb.rows_x + 255) / 256), fy = int((jb.rows_y + 255) / 256);
  // per-slot regions: gram units, reduce units, form units
  TRY(ensure_units(P, slot, jb.rows_x, jb.rows_y, s));
  LrUnit* du = P->units + int64_t(slot) * P->slot_units;
  ReduceUnit* dr = reinterpret_cast<ReduceUnit*>(du + P->cap_gram);
  LrUnit* dfu = du + P->cap_gram + 2;
  double* gp = P->gpart + int64_t(slot) * P->cap_gram * kG2;
  HFDE_LAUNCH(k_lr_gram, dim3(cx + cy), dim3(256), 0, s, jb, du, gp);
  HFDE_LAUNCH(k_gram_reduce, dim3(2), dim3(256), 0, s, dr, gp, P->grams);
  if (!recompress) {
    HFDE_LAUNCH(k_lr_frob, dim3(1), dim3(256), 0, s, jb, P->grams, P->frob + slot);
    return HODLR_OK;
  }
  HFDE_LAUNCH(k_lr_core, dim3(1), dim3(kCoreWG), kFactorLdsBytes, s, jb, P->grams, P->mbuf);
  HFDE_LAUNCH(k_lr_form, dim3(fx + fy), dim3(256), 0, s, jb, dfu, P->mbuf);
  return HODLR_OK;
}

// Device-to-host reads of the step's control values go through pinned host
// memory (an asynchronous copy, then one wait), not through a pageable buffer.
hodlr_status read_ranks(fde2d_plan P, int32_t* h, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(P->host_ranks, P->ranks, kR_N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  memcpy(h, P->host_ranks, kR_N * sizeof(int32_t));
  return HODLR_OK;
}

hodlr_status read_frob(fde2d_plan P, int slot, double* v, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(P->host_frob, P->frob + slot, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *v = *P->host_frob;
  return HODLR_OK;
}

void copy_cols(int64_t rows, const int32_t* rdev, int rfix, const double* src, int64_t lds, double* dst, int64_t ldd,
               double sc, hipStream_t s) {
  const int blocks = int(std::min<int64_t>((rows * 64 + 255) / 256, 4096));
  HFDE_LAUNCH(k_copy_cols, dim3(blocks), dim3(256), 0, s, rows, rdev, rfix, src, lds, dst, ldd, sc);
}

// dst = sc * E src on cols columns (E = mass (I + mc (S + S^T))).
void mass_cols(int64_t rows, int cols, double mass, double mc, const double* src, int64_t lds, double* dst,
               int64_t ldd, double sc, hipStream_t s) {
  if (cols <= 0) return;
  const int blocks = int(std::min<int64_t>((rows * cols + 255) / 256, 4096));
  HFDE_LAUNCH(k_mass_cols, dim3(blocks), dim3(256), 0, s, rows, cols, mass, mc, src, lds, dst, ldd, sc);
}

// ||S||_F of a sum of low-rank products formed entry by entry (k_lrs_dense).
hodlr_status dense_norm(fde2d_plan P, const LrSum& S, double& norm, hipStream_t s) {
  const dim3 grid(unsigned((P->nx + 63) / 64), unsigned((P->ny + 63) / 64));
  int K = 0;
  for (int g = 0; g < S.ng; ++g) K += S.g[g].cfix;    // every caller passes host column counts
  P->lrs_flops += 2.0 * double(P->nx) * double(P->ny) * K;
  HFDE_LAUNCH(k_lrs_dense, grid, dim3(256), 0, s, S, P->lrs_part);
  HFDE_LAUNCH(k_sum_partials, dim3(1), dim3(256), 0, s, P->lrs_part, int64_t(grid.x) * grid.y, P->dnorm);
  HIP_TRY(hipMemcpyAsync(P->host_frob + 1, P->dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  norm = std::sqrt(std::max(P->host_frob[1], 0.0));
  return HODLR_OK;
}

// Low-rank approximation of a sum S = sum_g s_g P_g Q_g^T by a randomized
// range finder on its factors (S is never formed): Y = S Om with a
// kSketch-column uniform Om (counter-based generator, seed), two
// orthonormalising passes (Q1 from Y, Q2 from Q1), B = S^T Q2, then Q2 B^T
// recompressed at tau_rel ||S||_F and at most rmax columns into (U, V), rank
// at *rank_out.
hodlr_status compress_lrsum(fde2d_plan P, const LrSum& S, double tau_rel, uint64_t seed, int rmax, double* U,
                            int64_t ldu, double* V, int64_t ldv, int32_t* rank_out, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny;
  constexpr int kSk = kSketch;
  static_assert(kSk == kLrsK, "sketch width");
  HFDE_LAUNCH(k_fill_uniform, dim3(256), dim3(256), 0, s, P->om, ny * kSk, seed);
  const unsigned sy = unsigned((ny + kLrsSlice - 1) / kLrsSlice), sx = unsigned((nx + kLrsSlice - 1) / kLrsSlice);
  const unsigned tb = unsigned((kLrsCols * kLrsK + 255) / 256);
  HFDE_LAUNCH(k_lrs_cross, dim3(sy), dim3(256), 0, s, S, 0, P->om, ny, kSk, P->lrs_cpart);
  HFDE_LAUNCH(k_lrs_cross_sum, dim3(tb), dim3(256), 0, s, P->lrs_cpart, int(sy), P->lrs_t);
  HFDE_LAUNCH(k_lrs_apply, dim3(unsigned((nx + 255) / 256)), dim3(256), 0, s, S, 0, P->lrs_t, kSk, P->sk_y, nx);
  HFDE_LAUNCH(k_set_identity, dim3((kSk * kSk + 255) / 256), dim3(256), 0, s, P->eye, kSk, kSk);
  for (int pass = 0; pass < 2; ++pass) {
    LrJob oj{};
    oj.X.g[0] = pass == 0 ? grp(P->sk_y, nx, nullptr, kSk, 1.0) : grp(P->sk_q1, nx, P->ranks + kR_Q1, 0, 1.0);
    oj.X.g[1] = oj.X.g[2] = grp_none();
    oj.Y.g[0] = pass == 0 ? grp(P->eye, kSk, nullptr, kSk, 1.0) : grp(P->eye, kSk, P->ranks + kR_Q1, 0, 1.0);
    oj.Y.g[1] = oj.Y.g[2] = grp_none();
    oj.rows_x = nx;
    oj.rows_y = kSk;
    oj.rank_out = P->ranks + (pass == 0 ? kR_Q1 : kR_Q2);
    oj.tau = 0.0;
    oj.tau_rel = 1e-15;
    oj.rmax = kSk;
    oj.U = pass == 0 ? P->sk_q1 : P->sk_q2;
    oj.ldu = nx;
    oj.V = P->sk_junk;
    oj.ldv = kSk;
    TRY(run_lr(P, oj, 10 + pass, true, s));
  }
  HFDE_LAUNCH(k_lrs_cross, dim3(sx), dim3(256), 0, s, S, 1, P->sk_q2, nx, kSk, P->lrs_cpart);
  HFDE_LAUNCH(k_lrs_cross_sum, dim3(tb), dim3(256), 0, s, P->lrs_cpart, int(sx), P->lrs_t);
  HFDE_LAUNCH(k_lrs_apply, dim3(unsigned((ny + 255) / 256)), dim3(256), 0, s, S, 1, P->lrs_t, kSk, P->sk_b, ny);
  LrJob tj{};
  tj.X.g[0] = grp(P->sk_q2, nx, P->ranks + kR_Q2, 0, 1.0);
  tj.X.g[1] = tj.X.g[2] = grp_none();
  tj.Y.g[0] = grp(P->sk_b, ny, P->ranks + kR_Q2, 0, 1.0);
  tj.Y.g[1] = tj.Y.g[2] = grp_none();
  tj.rows_x = nx;
  tj.rows_y = ny;
  tj.rank_out = rank_out;
  tj.tau = 0.0;
  tj.tau_rel = tau_rel;
  tj.rmax = rmax;
  tj.U = U;
  tj.ldu = ldu;
  tj.V = V;
  tj.ldv = ldv;
  TRY(run_lr(P, tj, 12, true, s));
  return HODLR_OK;
}

// Low-rank approximation of a dense FP32 nx x ny matrix X (ld nx) by a
// randomized range finder: Y = X Om with a kSketch-column uniform Om
// (counter-based generator, seed), two orthonormalising passes (Q1 from Y,
// Q2 from Q1), B = X^T Q2, then Q2 B^T recompressed at tau_rel ||X||_F and at
// most rmax columns into (U, V), rank at *rank_out.
hodlr_status compress_dense(fde2d_plan P, const float* X, double tau_rel, uint64_t seed, int rmax, double* U,
                            int64_t ldu, double* V, int64_t ldv, int32_t* rank_out, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny;
  constexpr int kSk = kSketch;
  HFDE_LAUNCH(k_fill_uniform, dim3(256), dim3(256), 0, s, P->om, ny * kSk, seed);
  HFDE_LAUNCH(k_field_times, dim3(unsigned((nx + 255) / 256)), dim3(256), 0, s, nx, ny, X, P->om, kSk, P->sk_y);
  HFDE_LAUNCH(k_set_identity, dim3((kSk * kSk + 255) / 256), dim3(256), 0, s, P->eye, kSk, kSk);
  for (int pass = 0; pass < 2; ++pass) {
    LrJob oj{};
    oj.X.g[0] = pass == 0 ? grp(P->sk_y, nx, nullptr, kSk, 1.0) : grp(P->sk_q1, nx, P->ranks + kR_Q1, 0, 1.0);
    oj.X.g[1] = oj.X.g[2] = grp_none();
    oj.Y.g[0] = pass == 0 ? grp(P->eye, kSk, nullptr, kSk, 1.0) : grp(P->eye, kSk, P->ranks + kR_Q1, 0, 1.0);
    oj.Y.g[1] = oj.Y.g[2] = grp_none();
    oj.rows_x = nx;
    oj.rows_y = kSk;
    oj.rank_out = P->ranks + (pass == 0 ? kR_Q1 : kR_Q2);
    oj.tau = 0.0;
    oj.tau_rel = 1e-15;
    oj.rmax = kSk;
    oj.U = pass == 0 ? P->sk_q1 : P->sk_q2;
    oj.ldu = nx;
    oj.V = P->sk_junk;                         // unused right factor (kSk x r)
    oj.ldv = kSk;
    TRY(run_lr(P, oj, 10 + pass, true, s));
  }
  HFDE_LAUNCH(k_field_t_times, dim3(unsigned((ny + 255) / 256)), dim3(256), 0, s, nx, ny, X, P->sk_q2,
              P->ranks + kR_Q2, P->sk_b);
  LrJob tj{};
  tj.X.g[0] = grp(P->sk_q2, nx, P->ranks + kR_Q2, 0, 1.0);
  tj.X.g[1] = tj.X.g[2] = grp_none();
  tj.Y.g[0] = grp(P->sk_b, ny, P->ranks + kR_Q2, 0, 1.0);
  tj.Y.g[1] = tj.Y.g[2] = grp_none();
  tj.rows_x = nx;
  tj.rows_y = ny;
  tj.rank_out = rank_out;
  tj.tau = 0.0;
  tj.tau_rel = tau_rel;
  tj.rmax = rmax;
  tj.U = U;
  tj.ldu = ldu;
  tj.V = V;
  tj.ldv = ldv;
  TRY(run_lr(P, tj, 12, true, s));
  return HODLR_OK;
}

// Shift pairs 4b .. min(4b + 4, J) - 1 of a sweep, main chain: solves of nc
// columns and the residual update G -= w Z, H -= w Y, then the Gram norm of
// the residual G H^T into frob slot 1.  Every column count is read on the
// device, so the same launches serve any right-hand-side rank up to nc.
hodlr_status enqueue_main_block(fde2d_plan P, int b, int nc, hipStream_t s) {
  hodlr_mat m = P->mat;
  const int64_t nx = P->nx, ny = P->ny, tn = m->total_n;
  const MassPair E{P->mass_x, P->mc_x, P->mass_y, P->mc_y};
  const int jend = std::min(4 * b + 4, P->J);
  for (int jo = 4 * b; jo < jend; ++jo) {
    const int j = P->order[jo];
    const Item& ix = m->items[j];
    const Item& iy = m->items[P->J + j];
    if (jo == 4 * b) {       // the block's first pair: G, H into its rows of the workspace
      copy_cols(nx, P->ranks + kR_R0, 0, P->G, nx, P->xin + ix.row0, tn, 1.0, s);
      copy_cols(ny, P->ranks + kR_R0, 0, P->H, ny, P->xin + iy.row0, tn, 1.0, s);
    } else {                 // the previous pair's update, writing the new G, H into this pair's rows too
      const int jp = P->order[jo - 1];
      const Item& px = m->items[jp];
      const Item& py = m->items[P->J + jp];
      HFDE_LAUNCH(k_adi_update_copy, dim3(256), dim3(256), 0, s, nx, ny, P->ranks + kR_R0, P->p[jp] + P->q[jp],
                  P->xin + px.row0, tn, P->xin + py.row0, tn, P->G, nx, P->H, ny, P->xin + ix.row0,
                  P->xin + iy.row0, tn, E);
    }
    launch_solve_units(m, m->opts.prec, P->pair_wu + P->pwu_off[j], P->pwu_cnt[j], P->pair_nu + P->pnu_off[j],
                       P->pnu_cnt[j], P->xin, tn, P->xin, tn, nc, s);
    if (jo + 1 == jend) {    // the block's last pair: its update alone (the block's norm reads G, H)
      const double w = P->p[j] + P->q[j];
      HFDE_LAUNCH(k_adi_update, dim3(256), dim3(256), 0, s, nx, ny, P->ranks + kR_R0, w, P->xin + ix.row0, tn,
                  P->xin + iy.row0, tn, P->G, nx, P->H, ny, E);
    }
  }
  LrJob nj{};
  nj.X.g[0] = grp(P->G, nx, P->ranks + kR_R0, 0, 1.0);
  nj.X.g[1] = nj.X.g[2] = grp_none();
  nj.Y.g[0] = grp(P->H, ny, P->ranks + kR_R0, 0, 1.0);
  nj.Y.g[1] = nj.Y.g[2] = grp_none();
  nj.rows_x = nx;
  nj.rows_y = ny;
  return run_lr(P, nj, 1, false, s);
}

// The same shift pairs, accumulation chains: D_g <- recompress([D_g, w Z_j][W_g, Y_j])
// for the pairs jo with jo mod 2 = g (D_0 in Zd/Wd, D_1 in Ze/We, each
// ping-ponging between its two buffers; work slots 2, 3 and 13, 14).  Z_j,
// Y_j are the solve outputs in shift j's own rows of the workspace, which no
// other shift of the sweep touches, so the chains run beside the solves.
hodlr_status enqueue_d_block(fde2d_plan P, int b, int g, hipStream_t s) {
  hodlr_mat m = P->mat;
  const int64_t nx = P->nx, ny = P->ny, tn = m->total_n;
  const double tol = P->opts.tol;
  double* const* Zg = g == 0 ? P->Zd : P->Ze;
  double* const* Wg = g == 0 ? P->Wd : P->We;
  const int rk = g == 0 ? kR_D0 : kR_E0;
  for (int jo = 4 * b + g; jo < std::min(4 * b + 4, P->J); jo += 2) {
    const int j = P->order[jo];
    const int parity = (jo >> 1) & 1;
    const Item& ix = m->items[j];
    const Item& iy = m->items[P->J + j];
    const double w = P->p[j] + P->q[j];
    LrJob jb{};
    jb.X.g[0] = grp(Zg[parity], nx, P->ranks + rk + parity, 0, 1.0);
    jb.X.g[1] = grp(P->xin + ix.row0, tn, P->ranks + kR_R0, 0, w);
    jb.X.g[2] = grp_none();
    jb.Y.g[0] = grp(Wg[parity], ny, P->ranks + rk + parity, 0, 1.0);
    jb.Y.g[1] = grp(P->xin + iy.row0, tn, P->ranks + kR_R0, 0, 1.0);
    jb.Y.g[2] = grp_none();
    jb.rows_x = nx;
    jb.rows_y = ny;
    jb.rank_out = P->ranks + rk + (1 - parity);
    jb.tau = 0.0;
    jb.tau_rel = 0.1 * tol;
    jb.rmax = kRS;
    jb.U = Zg[1 - parity];
    jb.ldu = nx;
    jb.V = Wg[1 - parity];
    jb.ldv = ny;
    TRY(run_lr(P, jb, (g == 0 ? 2 : 13) + parity, true, s));
  }
  return HODLR_OK;
}

// Capture `enqueue` on stream s into ge (once), then replay it.
template <typename F>
hodlr_status replay(hipGraphExec_t& ge, hipStream_t s, F&& enqueue) {
  if (!ge) {
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hodlr_status st = enqueue();
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (st != HODLR_OK) return st;
    HIP_TRY(ec);
    const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(ei);
  }
  HIP_TRY(hipGraphLaunch(ge, s));
  return HODLR_OK;
}

// One fADI sweep on the right-hand side G H^T (rank r0, in P->G / P->H; they are
// consumed).  Accumulates the sweep's solution into Zd/Wd; returns the steps
// taken and the parity holding the result.  The convergence test (fADI
// residual ||G_J H_J^T||_F <= target) comes after every block of four shift
// pairs.  The solution accumulates in two chains
// (even and odd shift pairs) that are merged at the end.  On a stream of its
// own (and without kernel timing) each block's solves and each chain are HIP
// graphs captured on first use, and the two chains run on two more streams
// one block behind the solves, joined before the merge; otherwise everything
// runs in the same order on one stream.
hodlr_status adi_sweep(fde2d_plan P, int r0, double target, int& steps, int& parity, hipStream_t s) {
  const double tol = P->opts.tol;
  const int64_t nx = P->nx, ny = P->ny;
  HIP_TRY(hipMemsetAsync(P->ranks + kR_D0, 0, sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P->ranks + kR_E0, 0, sizeof(int32_t), s));
  parity = 0;
  steps = 0;
  if (r0 == 0) return HODLR_OK;
  const int wide = r0 > kNCS ? 1 : 0;
  const int nc = wide ? 2 * kNCS : kNCS;
  const bool graphs = s != nullptr && g_timer == nullptr && P->side[0] != nullptr;
  if (graphs)
    for (int slot : {1, 2, 3, 13, 14}) TRY(ensure_units(P, slot, nx, ny, s));
  const int nb = (P->J + 3) / 4;
  hodlr_status res = HODLR_OK;
  for (int b = 0; b < nb && res == HODLR_OK; ++b) {
    if (graphs) {
      res = replay(P->blk_graph[wide][b], s, [&] { return enqueue_main_block(P, b, nc, s); });
      if (res != HODLR_OK) break;
      HIP_TRY(hipEventRecord(P->ev_blk, s));
      for (int g = 0; g < 2 && res == HODLR_OK; ++g) {
        if (4 * b + g >= P->J) continue;         // no pair of this chain in the block
        HIP_TRY(hipStreamWaitEvent(P->side[g], P->ev_blk, 0));
        res = replay(P->d_graph[g][b], P->side[g], [&] { return enqueue_d_block(P, b, g, P->side[g]); });
      }
      if (res != HODLR_OK) break;
    } else {
      TRY(enqueue_main_block(P, b, nc, s));
      TRY(enqueue_d_block(P, b, 0, s));
      TRY(enqueue_d_block(P, b, 1, s));
    }
    steps = std::min(4 * b + 4, P->J);
    double f2 = 0.0;
    res = read_frob(P, 1, &f2, s);
    if (res != HODLR_OK || std::sqrt(std::max(f2, 0.0)) <= target) break;
  }
  if (graphs) {                                  // join the accumulation chains
    for (int g = 0; g < 2; ++g) {
      HIP_TRY(hipEventRecord(P->ev_done[g], P->side[g]));
      HIP_TRY(hipStreamWaitEvent(s, P->ev_done[g], 0));
    }
  }
  if (res != HODLR_OK) return res;
  // chain g took n_g = ceil or floor of steps / 2 pairs; its result is in buffer n_g & 1
  const int p0 = ((steps + 1) / 2) & 1, p1 = (steps / 2) & 1;
  parity = p0;
  if (steps < 2) return HODLR_OK;
  LrJob mj{};                                    // D <- recompress([D_0, D_1][W_0, W_1])
  mj.X.g[0] = grp(P->Zd[p0], nx, P->ranks + kR_D0 + p0, 0, 1.0);
  mj.X.g[1] = grp(P->Ze[p1], nx, P->ranks + kR_E0 + p1, 0, 1.0);
  mj.X.g[2] = grp_none();
  mj.Y.g[0] = grp(P->Wd[p0], ny, P->ranks + kR_D0 + p0, 0, 1.0);
  mj.Y.g[1] = grp(P->We[p1], ny, P->ranks + kR_E0 + p1, 0, 1.0);
  mj.Y.g[2] = grp_none();
  mj.rows_x = nx;
  mj.rows_y = ny;
  mj.rank_out = P->ranks + kR_D0 + (1 - p0);
  mj.tau = 0.0;
  mj.tau_rel = 0.1 * tol;
  mj.rmax = kRS;
  mj.U = P->Zd[1 - p0];
  mj.ldu = nx;
  mj.V = P->Wd[1 - p0];
  mj.ldv = ny;
  TRY(run_lr(P, mj, 15, true, s));
  parity = 1 - p0;
  return HODLR_OK;
}


// ---------------------------------------------------------------------------
// Extended Krylov solver of A D + D B^T = G H^T (Sec. 4.3), in place of an
// fADI sweep: orthonormal bases U of EK(A, G) = span{G, A^-1 G, A G,
// A^-2 G, ...} and V of EK(B, H) are grown a block at a time (two extended
// block Arnoldi processes; the products with A and B are the exact Toeplitz
// products, the solves HODLR solves with the unshifted factors refined once
// against the exact product),
// the projected equation T_A Y + Y T_B^T = (U^T G)(V^T H)^T is solved, and
// D = U Y V^T.  A new block is orthogonalised against the basis by a block
// Gram-Schmidt pass and orthonormalised with its directions below 1e-10 of
// its norm before the pass dropped (deflation: the block shrinks once the
// space stops growing in a direction), then projected and orthonormalised
// once more.  The projected equation is solved by factored ADI on explicit
// inverses of T_A + q_j I and T_B + p_j I, with Zolotarev shift pairs of its
// own for the plan's spectral intervals.
// The residual of D = U Y V^T splits into three orthogonal terms,
// (A U - U T_A) Y V^T, U Y (B V - V T_B)^T and U (T_A Y + Y T_B^T - G' H'^T) V^T,
// whose norms are formed from explicit products (no Gram differences), so the
// test resolves the residual to about u ||A|| ||D||.

constexpr double kEkDrop = 1e-10;   // deflation level of a new block, relative to its norm
constexpr int kEkIterMax = 40;

struct EkSide {
  double* Q;        // n x kEkMax orthonormal basis
  double* AQ;       // the operator times it
  double* T;        // kEkMax x kEkMax projected operator Q^T (op Q)
  int64_t n;
  int m = 0;        // basis columns
  int o1 = 0, c1 = 0;   // the operator half's last block (columns o1 .. o1 + c1 - 1)
  int o2 = 0, c2 = 0;   // the inverse half's last block
};

// C = alpha op(A) op(B) + beta C (k_ek_gemm), the inner dimension split over
// work-groups when the output has few tiles.
hodlr_status ek_gemm(fde2d_plan P, int ta, int tb, int M, int N, int64_t K, double alpha, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s,
                     const int32_t* ndev = nullptr) {
  if (M <= 0 || N <= 0) return HODLR_OK;
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int64_t kchunk = std::max<int64_t>(K, 1);
  if (tiles < 128 && K >= 128) {
    int64_t ns = std::min<int64_t>({(K + 63) / 64, int64_t(kEkSplit), int64_t((256 + tiles - 1) / tiles)});
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, int64_t(kEkMax) * kEkMax / (int64_t(M) * N)));
    kchunk = ((K + ns - 1) / ns + 15) / 16 * 16;
  }
  const int nsplit = int(std::max<int64_t>(1, (K + kchunk - 1) / kchunk));
  P->ek_gemm_flops += 2.0 * double(M) * double(N) * double(K);
  HFDE_LAUNCH(k_ek_gemm, dim3(unsigned((M + 63) / 64), unsigned((N + 63) / 64), unsigned(nsplit)), dim3(256), 0, s,
              ta, tb, M, N, ndev, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, P->ekPart);
  if (nsplit > 1)
    HFDE_LAUNCH(k_ek_gemm_sum, dim3(unsigned(std::min<int64_t>((int64_t(M) * N + 255) / 256, 1024))), dim3(256), 0,
                s, M, N, ndev, nsplit, P->ekPart, alpha, beta, C, ldc);
  return HODLR_OK;
}

// ||X||_F^2 of an m x n block into ekNrm[slot] (device).
void ek_sumsq(fde2d_plan P, int64_t m, int n, const double* X, int64_t ld, int slot, hipStream_t s) {
  const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((m * n + 255) / 256, 512)));
  HFDE_LAUNCH(k_ek_sumsq, dim3(blocks), dim3(256), 0, s, m, std::max(n, 0), X, ld, P->ekPart);
  HFDE_LAUNCH(k_sum_partials, dim3(1), dim3(256), 0, s, P->ekPart, int64_t(blocks), P->ekNrm + slot);
}

// The solver's shift pairs and arrays: from the library's allocations, from
// the workspace given by fde2d_ek_attach_workspace, or (P->sizing) only
// counted in P->ws_used.
hodlr_status ek_alloc(fde2d_plan P) {
  const int64_t nx = P->nx, ny = P->ny, mr = std::max(nx, ny);
  const int64_t E2 = int64_t(kEkMax) * kEkMax;
  // the projected equation's shift pairs: as many as the intervals need for
  // opts.tol / 10, whatever cap the plan's shifted factor sets have
  int J = 1;
  for (; J < 64; ++J) {
    zolotarev_shifts(P->iv[0], P->iv[1], P->iv[2], P->iv[3], J, P->ek_p, P->ek_q);
    if (zolotarev_bound(P->iv[0], P->iv[1], P->iv[2], P->iv[3], P->ek_p, P->ek_q) <= 0.1 * P->opts.tol) break;
  }
  zolotarev_shifts(P->iv[0], P->iv[1], P->iv[2], P->iv[3], J, P->ek_p, P->ek_q);
  P->ek_J = J;
  bool ok = plan_alloc(P, &P->ekU, nx * kEkMax) == HODLR_OK && plan_alloc(P, &P->ekAU, nx * kEkMax) == HODLR_OK &&
            plan_alloc(P, &P->ekV, ny * kEkMax) == HODLR_OK && plan_alloc(P, &P->ekBV, ny * kEkMax) == HODLR_OK &&
            plan_alloc(P, &P->ekTA, E2) == HODLR_OK && plan_alloc(P, &P->ekTB, E2) == HODLR_OK &&
            plan_alloc(P, &P->ekW, mr * kRS) == HODLR_OK && plan_alloc(P, &P->ekO, mr * kRS) == HODLR_OK &&
            plan_alloc(P, &P->ekS, int64_t(kEkMax) * kRS) == HODLR_OK && plan_alloc(P, &P->ekPart, E2) == HODLR_OK &&
            plan_alloc(P, &P->ekShift, 2 * J) == HODLR_OK && plan_alloc(P, &P->ekLU, 2 * J * E2) == HODLR_OK &&
            plan_alloc(P, &P->ekInv, 2 * J * E2) == HODLR_OK &&
            plan_alloc(P, &P->ekPiv, int64_t(2) * J * kEkMax) == HODLR_OK &&
            plan_alloc(P, &P->ekFlag, 2 * J) == HODLR_OK;
  for (int k = 0; k < 2 && ok; ++k)
    ok = plan_alloc(P, &P->ekG[k], int64_t(kEkMax) * kRS) == HODLR_OK &&
         plan_alloc(P, &P->ekH[k], int64_t(kEkMax) * kRS) == HODLR_OK;
  ok = ok && plan_alloc(P, &P->ekKZ, int64_t(kEkMax) * J * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekKY, int64_t(kEkMax) * J * kRS) == HODLR_OK && plan_alloc(P, &P->ekY, E2) == HODLR_OK &&
       plan_alloc(P, &P->ekOm, int64_t(kEkMax) * kEkSk) == HODLR_OK &&
       plan_alloc(P, &P->ekYs, int64_t(kEkMax) * kEkSk) == HODLR_OK &&
       plan_alloc(P, &P->ekQ1, int64_t(kEkMax) * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekQ2, int64_t(kEkMax) * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekBt, int64_t(kEkMax) * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekEye, kEkSk * kEkSk) == HODLR_OK && plan_alloc(P, &P->ekZf, nx * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekWf, ny * kRS) == HODLR_OK && plan_alloc(P, &P->ekJunk, kEkSk * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekG0, int64_t(kEkMax) * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekH0, int64_t(kEkMax) * kRS) == HODLR_OK && plan_alloc(P, &P->ekR, mr * kEkMax) == HODLR_OK &&
       plan_alloc(P, &P->ekY1, E2) == HODLR_OK && plan_alloc(P, &P->ekRs, E2) == HODLR_OK &&
       plan_alloc(P, &P->ekNrm, 4) == HODLR_OK && plan_alloc(P, &P->ekPivX, nx) == HODLR_OK &&
       plan_alloc(P, &P->ekPivY, ny) == HODLR_OK && plan_alloc(P, &P->ekGt, nx * kRS) == HODLR_OK &&
       plan_alloc(P, &P->ekHt, ny * kRS) == HODLR_OK;
  if (!ok) return P->ws ? HODLR_EWORKSPACE : HODLR_ENOMEM;
  return HODLR_OK;
}

// Arrays of the solver (first use), the shifts on the device, and the
// factorisation of the unshifted A and B (the batch of the exact products).
hodlr_status ek_prepare(fde2d_plan P, hipStream_t s) {
  if (P->ek_ready) return HODLR_OK;
  if (P->ws && !P->ek_ws) return HODLR_EWORKSPACE;    // a workspace plan needs fde2d_ek_attach_workspace
  TRY(ek_alloc(P));
  const int64_t nx = P->nx, ny = P->ny;
  const int J = P->ek_J;
  // pivots of the mass matrices' tridiagonal LU: m_0 = 1, m_i = 1 - mc^2 / m_{i-1}
  for (int side = 0; side < 2; ++side) {
    const double mc = side == 0 ? P->mc_x : P->mc_y;
    const int64_t n = side == 0 ? nx : ny;
    std::vector<double> piv(n, 1.0);
    for (int64_t i = 1; i < n; ++i) piv[i] = 1.0 - mc * mc / piv[i - 1];
    HIP_TRY(hipMemcpy(side == 0 ? P->ekPivX : P->ekPivY, piv.data(), n * sizeof(double), hipMemcpyHostToDevice));
  }
  std::vector<double> sh(2 * J);
  for (int j = 0; j < J; ++j) {
    sh[j] = P->ek_q[j];
    sh[J + j] = P->ek_p[j];
  }
  HIP_TRY(hipMemcpyAsync(P->ekShift, sh.data(), sh.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HFDE_LAUNCH(k_set_identity, dim3((kEkSk * kEkSk + 255) / 256), dim3(256), 0, s, P->ekEye, kEkSk, kEkSk);
  HFDE_LAUNCH(k_fill_uniform, dim3(64), dim3(256), 0, s, P->ekOm, int64_t(kEkMax) * kEkSk, uint64_t(0xe4e4));
  HIP_TRY(hipStreamSynchronize(s));
  hodlr_info fi{};
  const hodlr_status st = hodlr_factor(P->ctx, P->exact, &fi);
  if (st != HODLR_OK && st != HODLR_ERANK) return st;
  P->ek_ready = true;
  return HODLR_OK;
}

// Y = E^-1 X on `cols` columns of one side (0: x, 1: y); a copy for an identity E.
void ek_mass_solve(fde2d_plan P, int side, int cols, const double* X, int64_t ldx, double* Y, int64_t ldy,
                   hipStream_t s) {
  const double mass = side == 0 ? P->mass_x : P->mass_y, mc = side == 0 ? P->mc_x : P->mc_y;
  const int64_t n = side == 0 ? P->nx : P->ny;
  if (cols <= 0) return;
  if (mc == 0.0 && mass == 1.0) {
    copy_cols(n, nullptr, cols, X, ldx, Y, ldy, 1.0, s);
    return;
  }
  HFDE_LAUNCH(k_ek_mass_solve, dim3(unsigned((n + kMsTile - 1) / kMsTile), unsigned(cols)), dim3(256), 0, s, n,
              mass, mc, side == 0 ? P->ekPivX : P->ekPivY, X, ldx, Y, ldy);
}

// Enqueue the append of the c-column candidate block in ekW (ld n) to the
// side's basis (side 0: A, 1: B): a block Gram-Schmidt pass, an
// orthonormalisation that drops the directions below kEkDrop times the
// block's norm before the pass (read on the device), one more pass and a
// final orthonormalisation into the basis columns S.m ..; the number of new
// columns lands in ranks[kR_EK2] (side 0) or ranks[kR_EK4] (side 1).  Nothing
// waits for the device: ek_add_pair reads both counts.
hodlr_status ek_add(fde2d_plan P, const EkSide& S, int c, int side, hipStream_t s) {
  const int64_t n = S.n;
  const int sl1 = side ? 20 : 16, sl2 = side ? 21 : 17;
  int32_t* rk1 = P->ranks + (side ? kR_EK3 : kR_EK1);
  int32_t* rk2 = P->ranks + (side ? kR_EK4 : kR_EK2);
  LrJob fj{};
  fj.X.g[0] = grp(P->ekW, n, nullptr, c, 1.0);
  fj.X.g[1] = fj.X.g[2] = grp_none();
  fj.Y.g[0] = grp(P->ekEye, kEkSk, nullptr, c, 1.0);
  fj.Y.g[1] = fj.Y.g[2] = grp_none();
  fj.rows_x = n;
  fj.rows_y = kEkSk;
  TRY(run_lr(P, fj, sl1, false, s));                  // ||W||_F^2 into frob[sl1]
  if (S.m > 0) {
    TRY(ek_gemm(P, 1, 0, S.m, c, n, 1.0, S.Q, n, P->ekW, n, 0.0, P->ekS, kEkMax, s));    // Q^T W
    TRY(ek_gemm(P, 0, 0, int(n), c, S.m, -1.0, S.Q, n, P->ekS, kEkMax, 1.0, P->ekW, n, s));   // W -= Q (Q^T W)
  }
  LrJob oj{};
  oj.X.g[0] = grp(P->ekW, n, nullptr, c, 1.0);
  oj.X.g[1] = oj.X.g[2] = grp_none();
  oj.Y.g[0] = grp(P->ekEye, kEkSk, nullptr, c, 1.0);
  oj.Y.g[1] = oj.Y.g[2] = grp_none();
  oj.rows_x = n;
  oj.rows_y = kEkSk;
  oj.rank_out = rk1;
  oj.tau = 0.0;
  oj.tau_rel = 0.0;
  oj.tau_sq = P->frob + sl1;
  oj.tau_sq_scale = kEkDrop;
  oj.rmax = std::min(kRS, kEkMax - S.m);
  oj.U = P->ekO;
  oj.ldu = n;
  oj.V = P->ekJunk;
  oj.ldv = kEkSk;
  TRY(run_lr(P, oj, sl1, true, s));
  if (S.m > 0) {
    TRY(ek_gemm(P, 1, 0, S.m, c, n, 1.0, S.Q, n, P->ekO, n, 0.0, P->ekS, kEkMax, s, rk1));
    TRY(ek_gemm(P, 0, 0, int(n), c, S.m, -1.0, S.Q, n, P->ekS, kEkMax, 1.0, P->ekO, n, s, rk1));
  }
  LrJob qj{};
  qj.X.g[0] = grp(P->ekO, n, rk1, 0, 1.0);
  qj.X.g[1] = qj.X.g[2] = grp_none();
  qj.Y.g[0] = grp(P->ekEye, kEkSk, rk1, 0, 1.0);
  qj.Y.g[1] = qj.Y.g[2] = grp_none();
  qj.rows_x = n;
  qj.rows_y = kEkSk;
  qj.rank_out = rk2;
  qj.tau = 0.0;
  qj.tau_rel = 1e-6;
  qj.rmax = std::min(kRS, kEkMax - S.m);
  qj.U = S.Q + int64_t(S.m) * n;
  qj.ldu = n;
  qj.V = P->ekJunk;
  qj.ldv = kEkSk;
  return run_lr(P, qj, sl2, true, s);
}

// Append candidate blocks to both bases: A's from srcA (ca columns, ld
// lda), B's from srcB; one wait for the two new column counts.
hodlr_status ek_add_pair(fde2d_plan P, EkSide& A, const double* srcA, int64_t lda, int ca, EkSide& B,
                         const double* srcB, int64_t ldb, int cb, int& added_a, int& added_b, hipStream_t s) {
  added_a = added_b = 0;
  const bool da = ca > 0 && A.m < kEkMax, db = cb > 0 && B.m < kEkMax;
  if (da) {
    copy_cols(A.n, nullptr, ca, srcA, lda, P->ekW, A.n, 1.0, s);
    TRY(ek_add(P, A, ca, 0, s));
  }
  if (db) {
    copy_cols(B.n, nullptr, cb, srcB, ldb, P->ekW, B.n, 1.0, s);
    TRY(ek_add(P, B, cb, 1, s));
  }
  if (!da && !db) return HODLR_OK;
  int32_t hr[kR_N];
  TRY(read_ranks(P, hr, s));
  if (da) added_a = hr[kR_EK2];
  if (db) added_b = hr[kR_EK4];
  A.m += added_a;
  B.m += added_b;
  return HODLR_OK;
}

// Products with the operators of the columns a0 .. A.m - 1 and b0 .. B.m - 1
// (exact Toeplitz products of both sides in one call), and the new rows and
// columns of T_A and T_B.
hodlr_status ek_products(fde2d_plan P, EkSide& A, int a0, EkSide& B, int b0, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny, ld = nx + ny;
  const int ca = A.m - a0, cb = B.m - b0, c = std::max(ca, cb);
  if (c == 0) return HODLR_OK;
  copy_cols(nx, nullptr, ca, A.Q + int64_t(a0) * nx, nx, P->ex_in, ld, 1.0, s);
  copy_cols(ny, nullptr, cb, B.Q + int64_t(b0) * ny, ny, P->ex_in + nx, ld, 1.0, s);
  launch_fft_matvec(P->exact, P->ex_in, ld, P->ex_out, ld, nullptr, 0, c, s);
  // finite elements: E_x^-1 A, E_y^-1 B (differences: copies)
  ek_mass_solve(P, 0, ca, P->ex_out, ld, A.AQ + int64_t(a0) * nx, nx, s);
  ek_mass_solve(P, 1, cb, P->ex_out + nx, ld, B.AQ + int64_t(b0) * ny, ny, s);
  for (int side = 0; side < 2; ++side) {
    EkSide& S = side == 0 ? A : B;
    const int m0 = side == 0 ? a0 : b0, m1 = S.m;
    if (m1 == m0) continue;
    const int64_t n = S.n;
    TRY(ek_gemm(P, 1, 0, m1, m1 - m0, n, 1.0, S.Q, n, S.AQ + int64_t(m0) * n, n, 0.0, S.T + int64_t(m0) * kEkMax,
                kEkMax, s));
    if (m0 > 0)
      TRY(ek_gemm(P, 1, 0, m1 - m0, m0, n, 1.0, S.Q + int64_t(m0) * n, n, S.AQ, n, 0.0, S.T + m0, kEkMax, s));
  }
  return HODLR_OK;
}

// The inverse half of an iteration: A^-1 and B^-1 (HODLR solves with the
// unshifted factors, refined) on the given blocks, appended to the bases.
hodlr_status ek_inverse_half(fde2d_plan P, EkSide& A, int ao, int ac, EkSide& B, int bo, int bc, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny, ld = nx + ny;
  const int c = std::max(ac, bc), a0 = A.m, b0 = B.m;
  int added_a = 0, added_b = 0;
  if (c > 0) {
    // b = E v (finite elements: (E^-1 A)^-1 = A^-1 E)
    mass_cols(nx, ac, P->mass_x, P->mc_x, A.Q + int64_t(ao) * nx, nx, P->ex_in, ld, 1.0, s);
    mass_cols(ny, bc, P->mass_y, P->mc_y, B.Q + int64_t(bo) * ny, ny, P->ex_in + nx, ld, 1.0, s);
    // x = M^-1 b with the stored factors, then refinement steps x += M^-1 (b - M x)
    // (exact products): the plain solve's error (about the factors'
    // precision times the condition) would perturb the inverse half of the basis
    hodlr_mat mx = P->exact;
    launch_solve(mx, mx->opts.prec, P->ex_in, ld, P->ex_out, ld, c, s);
    const int refine = mx->opts.prec == HODLR_MIXED_BF16 ? 2 : 1;
    double* r = P->ekR;
    double* d = P->ekR + ld * kRS;
    for (int k = 0; k < refine; ++k) {
      launch_fft_matvec(mx, P->ex_out, ld, r, ld, P->ex_in, ld, c, s);          // r = b - M x
      launch_solve(mx, mx->opts.prec, r, ld, d, ld, c, s);
      launch_axpby(ld, c, 1.0, d, ld, 1.0, P->ex_out, ld, P->ex_out, ld, s);
    }
    TRY(ek_add_pair(P, A, P->ex_out, ld, ac, B, P->ex_out + nx, ld, bc, added_a, added_b, s));
  }
  A.o2 = a0;
  A.c2 = added_a;
  B.o2 = b0;
  B.c2 = added_b;
  return ek_products(P, A, a0, B, b0, s);
}

// The projected equation on the current bases: U^T G, V^T H, the LU
// factors and inverses of the 2 ek_J shifted projected matrices, the projected
// fADI over those shift pairs (K_Z, K_Y), Y = K_Z K_Y^T, and the norm of the
// residual of U Y V^T (three orthogonal terms).
hodlr_status ek_projected(fde2d_plan P, const EkSide& A, const EkSide& B, const double* G, const double* H, int r0,
                          double& rn, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny;
  const int mA = A.m, mB = B.m, J = P->ek_J;
  const int64_t E2 = int64_t(kEkMax) * kEkMax;
  TRY(ek_gemm(P, 1, 0, mA, r0, nx, 1.0, A.Q, nx, G, nx, 0.0, P->ekG0, kEkMax, s));
  TRY(ek_gemm(P, 1, 0, mB, r0, ny, 1.0, B.Q, ny, H, ny, 0.0, P->ekH0, kEkMax, s));
  HFDE_LAUNCH(k_ek_lu, dim3(2 * J), dim3(kEkWG), 0, s, J, mA, A.T, mB, B.T, int64_t(kEkMax), P->ekShift, P->ekLU,
              int64_t(kEkMax), E2, P->ekPiv, P->ekFlag);
  HFDE_LAUNCH(k_ek_lu_inv, dim3(unsigned((std::max(mA, mB) + kEkInvCols - 1) / kEkInvCols), unsigned(2 * J)), dim3(256), 0, s, J, mA,
              mB, P->ekLU, int64_t(kEkMax), E2, P->ekPiv, P->ekInv, int64_t(kEkMax));
  const unsigned tiles = unsigned((mA + 15) / 16 + (mB + 15) / 16);
  const double* gin = P->ekG0;
  const double* hin = P->ekH0;
  for (int jo = 0; jo < J; ++jo) {
    const int j = jo;
    double* gout = P->ekG[jo & 1];
    double* hout = P->ekH[jo & 1];
    HFDE_LAUNCH(k_ek_adi_pair, dim3(tiles), dim3(256), 0, s, mA, mB, r0, P->ek_p[j] + P->ek_q[j], P->ekInv + j * E2,
                P->ekInv + (J + j) * E2, int64_t(kEkMax), gin, hin, gout, hout, P->ekKZ, P->ekKY, int64_t(kEkMax),
                jo * r0);
    gin = gout;
    hin = hout;
  }
  const int K = J * r0;
  TRY(ek_gemm(P, 0, 1, mA, mB, K, 1.0, P->ekKZ, kEkMax, P->ekKY, kEkMax, 0.0, P->ekY, kEkMax, s));
  // (A U) Y - U (T_A Y)
  TRY(ek_gemm(P, 0, 0, mA, mB, mA, 1.0, A.T, kEkMax, P->ekY, kEkMax, 0.0, P->ekY1, kEkMax, s));
  TRY(ek_gemm(P, 0, 0, int(nx), mB, mA, 1.0, A.AQ, nx, P->ekY, kEkMax, 0.0, P->ekR, nx, s));
  TRY(ek_gemm(P, 0, 0, int(nx), mB, mA, -1.0, A.Q, nx, P->ekY1, kEkMax, 1.0, P->ekR, nx, s));
  ek_sumsq(P, nx, mB, P->ekR, nx, 0, s);
  // (B V) Y^T - V (T_B Y^T)
  TRY(ek_gemm(P, 0, 1, mB, mA, mB, 1.0, B.T, kEkMax, P->ekY, kEkMax, 0.0, P->ekY1, kEkMax, s));
  TRY(ek_gemm(P, 0, 1, int(ny), mA, mB, 1.0, B.AQ, ny, P->ekY, kEkMax, 0.0, P->ekR, ny, s));
  TRY(ek_gemm(P, 0, 0, int(ny), mA, mB, -1.0, B.Q, ny, P->ekY1, kEkMax, 1.0, P->ekR, ny, s));
  ek_sumsq(P, ny, mA, P->ekR, ny, 1, s);
  // T_A Y + Y T_B^T - (U^T G)(V^T H)^T
  TRY(ek_gemm(P, 0, 0, mA, mB, mA, 1.0, A.T, kEkMax, P->ekY, kEkMax, 0.0, P->ekRs, kEkMax, s));
  TRY(ek_gemm(P, 0, 1, mA, mB, mB, 1.0, P->ekY, kEkMax, B.T, kEkMax, 1.0, P->ekRs, kEkMax, s));
  TRY(ek_gemm(P, 0, 1, mA, mB, r0, -1.0, P->ekG0, kEkMax, P->ekH0, kEkMax, 1.0, P->ekRs, kEkMax, s));
  ek_sumsq(P, mA, mB, P->ekRs, kEkMax, 2, s);
  HIP_TRY(hipMemcpyAsync(P->host_frob + 2, P->ekNrm, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  std::vector<int32_t> flags(2 * J);
  HIP_TRY(hipMemcpyAsync(flags.data(), P->ekFlag, flags.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int32_t f : flags)
    if (f) return HODLR_ESINGULAR;       // a shifted projected matrix had an exactly zero pivot
  rn = std::sqrt(std::max(P->host_frob[2] + P->host_frob[3] + P->host_frob[4], 0.0));
  return HODLR_OK;
}

// D = U Y V^T as low-rank factors: the range of Y from a kEkSk-column sketch
// (two orthonormalising passes, at most kRS columns), Z = U Q, W = V Y^T Q,
// recompressed at tol / 10 into Zd[0] / Wd[0] (rank at kR_D0).
hodlr_status ek_form(fde2d_plan P, const EkSide& A, const EkSide& B, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny;
  const int mA = A.m, mB = B.m;
  TRY(ek_gemm(P, 0, 0, mA, kEkSk, mB, 1.0, P->ekY, kEkMax, P->ekOm, kEkMax, 0.0, P->ekYs, kEkMax, s));
  for (int pass = 0; pass < 2; ++pass) {
    LrJob oj{};
    oj.X.g[0] = pass == 0 ? grp(P->ekYs, kEkMax, nullptr, kEkSk, 1.0) : grp(P->ekQ1, kEkMax, P->ranks + kR_EQ1, 0, 1.0);
    oj.X.g[1] = oj.X.g[2] = grp_none();
    oj.Y.g[0] = pass == 0 ? grp(P->ekEye, kEkSk, nullptr, kEkSk, 1.0) : grp(P->ekEye, kEkSk, P->ranks + kR_EQ1, 0, 1.0);
    oj.Y.g[1] = oj.Y.g[2] = grp_none();
    oj.rows_x = mA;
    oj.rows_y = kEkSk;
    oj.rank_out = P->ranks + (pass == 0 ? kR_EQ1 : kR_EQ2);
    oj.tau = 0.0;
    oj.tau_rel = 1e-15;
    oj.rmax = kRS;
    oj.U = pass == 0 ? P->ekQ1 : P->ekQ2;
    oj.ldu = kEkMax;
    oj.V = P->ekJunk;
    oj.ldv = kEkSk;
    TRY(run_lr(P, oj, 18 + pass, true, s));
  }
  int32_t hr[kR_N];
  TRY(read_ranks(P, hr, s));
  const int cq = hr[kR_EQ2];
  if (cq == 0) {
    HIP_TRY(hipMemsetAsync(P->ranks + kR_D0, 0, sizeof(int32_t), s));
    return HODLR_OK;
  }
  TRY(ek_gemm(P, 1, 0, mB, cq, mA, 1.0, P->ekY, kEkMax, P->ekQ2, kEkMax, 0.0, P->ekBt, kEkMax, s));
  TRY(ek_gemm(P, 0, 0, int(nx), cq, mA, 1.0, A.Q, nx, P->ekQ2, kEkMax, 0.0, P->ekZf, nx, s));
  TRY(ek_gemm(P, 0, 0, int(ny), cq, mB, 1.0, B.Q, ny, P->ekBt, kEkMax, 0.0, P->ekWf, ny, s));
  LrJob dj{};
  dj.X.g[0] = grp(P->ekZf, nx, nullptr, cq, 1.0);
  dj.X.g[1] = dj.X.g[2] = grp_none();
  dj.Y.g[0] = grp(P->ekWf, ny, nullptr, cq, 1.0);
  dj.Y.g[1] = dj.Y.g[2] = grp_none();
  dj.rows_x = nx;
  dj.rows_y = ny;
  dj.rank_out = P->ranks + kR_D0;
  dj.tau = 0.0;
  dj.tau_rel = 0.1 * P->opts.tol;
  dj.rmax = kRS;
  dj.capped = P->ranks + kR_CAP;
  dj.U = P->Zd[0];
  dj.ldu = nx;
  dj.V = P->Wd[0];
  dj.ldv = ny;
  return run_lr(P, dj, 15, true, s);
}

// Extended Krylov solve of A D + D B^T = G H^T (rank r0 in P->G / P->H),
// until the residual of U Y V^T is at most target; D in Zd[0] / Wd[0]
// (parity 0), steps = the iterations (each grows both bases by an operator
// block and an inverse block).  The projected equation is solved first one
// iteration before the count the last solve of the same kind (0: a step's
// first solve, 1: a correction) took, then where the residual's rate of
// decrease between the last two solves predicts the target (at most eight
// iterations on), or at the next iteration while there is no rate yet.
hodlr_status ek_solve(fde2d_plan P, int r0, double target, int kind, int& steps, int& parity, hipStream_t s) {
  const int64_t nx = P->nx, ny = P->ny;
  HIP_TRY(hipMemsetAsync(P->ranks + kR_D0, 0, sizeof(int32_t), s));
  parity = 0;
  steps = 0;
  if (r0 == 0) return HODLR_OK;
  if (r0 > kRS) return HODLR_EINVAL;
  TRY(ek_prepare(P, s));
  const bool verbose = getenv("HODLR_VERBOSE") != nullptr;
  EkSide A{P->ekU, P->ekAU, P->ekTA, nx}, B{P->ekV, P->ekBV, P->ekTB, ny};
  // finite elements: the equation E_x^-1 A D + D (E_y^-1 B)^T = (E_x^-1 G)(E_y^-1 H)^T
  const double* G = P->G;
  const double* H = P->H;
  if (P->fe) {
    ek_mass_solve(P, 0, r0, P->G, nx, P->ekGt, nx, s);
    ek_mass_solve(P, 1, r0, P->H, ny, P->ekHt, ny, s);
    G = P->ekGt;
    H = P->ekHt;
  }
  int added_a = 0, added_b = 0;
  TRY(ek_add_pair(P, A, G, nx, r0, B, H, ny, r0, added_a, added_b, s));
  A.c1 = added_a;
  B.c1 = added_b;
  TRY(ek_products(P, A, 0, B, 0, s));
  TRY(ek_inverse_half(P, A, A.o1, A.c1, B, B.o1, B.c1, s));
  int next = std::max(1, P->ek_last[kind] - 1), prev_it = 0, checks = 0;
  double prev_rn = -1.0, rn = 0.0;
  for (int it = 1;; ++it) {
    const bool full = A.m + 2 * kRS > kEkMax || B.m + 2 * kRS > kEkMax;
    const bool stuck = A.c1 + A.c2 + B.c1 + B.c2 == 0;
    const bool last = full || stuck || it >= kEkIterMax;
    if (it >= next || last) {
      TRY(ek_projected(P, A, B, G, H, r0, rn, s));
      ++checks;
      steps = it;
      if (rn <= target || last) break;
      int more = 1;
      if (prev_rn > 0.0 && rn < prev_rn) {
        const double rate = std::log(rn / prev_rn) / double(it - prev_it);   // log decrease per iteration
        more = int(std::ceil(std::log(target / rn) / rate));
        more = std::min(8, std::max(1, more));
      }
      prev_rn = rn;
      prev_it = it;
      next = it + more;
    }
    const int a0 = A.m, b0 = B.m;
    TRY(ek_add_pair(P, A, A.AQ + int64_t(A.o1) * nx, nx, A.c1, B, B.AQ + int64_t(B.o1) * ny, ny, B.c1, added_a,
                    added_b, s));
    A.o1 = a0;
    A.c1 = added_a;
    B.o1 = b0;
    B.c1 = added_b;
    TRY(ek_products(P, A, a0, B, b0, s));
    TRY(ek_inverse_half(P, A, A.o2, A.c2, B, B.o2, B.c2, s));
  }
  P->ek_last[kind] = steps;
  if (verbose)
    fprintf(stderr, "hodlr_fde: extended Krylov: %d iterations, bases %d x %d, %d projected solves, residual %.2e "
            "(target %.2e)\n", steps, A.m, B.m, checks, rn, target);
  return ek_form(P, A, B, s);
}

// One solve of the step: an fADI sweep, or the extended Krylov solver.
hodlr_status step_solve(fde2d_plan P, int r0, double target, int kind, int& steps, int& parity, hipStream_t s) {
  return P->use_ek ? ek_solve(P, r0, target, kind, steps, parity, s) : adi_sweep(P, r0, target, steps, parity, s);
}

}  // namespace

extern "C" {

void fde2d_plan_destroy(fde2d_plan p) {
  if (!p) return;
  for (hipStream_t sd : p->side)
    if (sd) (void)hipStreamSynchronize(sd);
  for (auto& row : p->blk_graph)
    for (hipGraphExec_t& ge : row)
      if (ge) (void)hipGraphExecDestroy(ge);
  for (auto& row : p->d_graph)
    for (hipGraphExec_t& ge : row)
      if (ge) (void)hipGraphExecDestroy(ge);
  if (p->ev_blk) (void)hipEventDestroy(p->ev_blk);
  for (hipEvent_t e : p->ev_done)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t sd : p->side)
    if (sd) (void)hipStreamDestroy(sd);
  hodlr_destroy(p->mat);
  hodlr_destroy(p->exact);
  for (void* q : p->allocs) (void)hipFree(q);
  if (p->host_ranks) (void)hipHostFree(p->host_ranks);
  delete p;
}

int fde2d_plan_shifts(fde2d_plan p, double* ps, double* qs, int cap) {
  if (!p) return 0;
  for (int j = 0; j < std::min(cap, p->J); ++j) {
    if (ps) ps[j] = p->p[j];
    if (qs) qs[j] = p->q[j];
  }
  return p->J;
}

// Shifts, shifted factor sets and work arrays of a 2D plan.  Modes as for
// the 1D build: library-allocated (ws == nullptr), carved from a caller's
// workspace, or sizing (need != nullptr: J is fixed from the coefficients as
// in a real plan, the two HODLR batches are sized by hodlr_workspace_size and
// the plan's own arrays counted; nothing is built).  The workspace holds the
// shifted batch, then the unshifted one, then the plan's arrays.
static hodlr_status plan2d_impl(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                                const hodlr_opts* hopts, const fde2d_opts* opts, void* ws, size_t ws_bytes,
                                fde2d_plan* out, size_t* need) {
  const bool sizing = need != nullptr;
  if (!opx) return set_arg(ctx, 2);
  if (!opy) return set_arg(ctx, 3);
  if (!hopts) return set_arg(ctx, 4);
  if (!opts || !(opts->tol > 0.0) || opts->max_shifts < 1 || opts->max_shifts > 64 || opts->max_rank < 1 ||
      opts->max_rank > kRS)
    return set_arg(ctx, 5);
  if (!sizing && !out) return set_arg(ctx, ws ? 8 : 6);
  if (opx->discretization != FDE_FD && opx->discretization != FDE_FE) return set_arg(ctx, 2);
  if (opy->discretization != FDE_FD && opy->discretization != FDE_FE) return set_arg(ctx, 3);
  hipStream_t s = ctx->stream;
  fde2d_plan P = new (std::nothrow) fde2d_plan_s;
  if (!P) return HODLR_ENOMEM;
  P->ctx = ctx;
  P->sizing = sizing;
  for (auto& u : P->unit_rows) u[0] = u[1] = -1;
  if (!sizing && hipHostMalloc(reinterpret_cast<void**>(&P->host_ranks), 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    P->host_ranks = nullptr;
    fde2d_plan_destroy(P);
    return HODLR_ENOMEM;
  }
  P->host_frob = reinterpret_cast<double*>(P->host_ranks + 32);
  // two more streams (default priority) for the sweeps' accumulation chains
  if (!sizing && s != nullptr && (hipStreamCreateWithFlags(&P->side[0], hipStreamNonBlocking) != hipSuccess ||
                       hipStreamCreateWithFlags(&P->side[1], hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreateWithFlags(&P->ev_blk, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&P->ev_done[0], hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&P->ev_done[1], hipEventDisableTiming) != hipSuccess)) {
    fde2d_plan_destroy(P);
    return HODLR_EHIP;
  }
  P->opts = *opts;
  P->nx = opx->n;
  P->ny = opy->n;
  P->shift_x = opx->shift;
  P->shift_y = opy->shift;
  // Spectral intervals [s, hi] of the pencils (A, E_x) and (B, E_y).
  // Differences (E = I): Gershgorin with sum_k |g_k| = 2 alpha, so
  // hi = s + 2 nu alpha max(d+ + d-).  Finite elements: a generalized
  // eigenvalue is s + nu v^H (D+ T + D- T^T) v / v^H E v; the stiffness form
  // is coercive for constant coefficients (real part >= 0), its magnitude is
  // at most ||D+ T + D- T^T||_2 |v|^2 <= (max d+ + max d-) sum_m |w_m| |v|^2,
  // and v^H E v >= |v|^2 / 3 (E's eigenvalues lie in (1/3, 1)).  The weights
  // are positive from w_3 on and w_0 > 0, w_1 < 0 and sum to zero, so
  // sum |w_m| = -2 (w_1 + min(w_2, 0)).
  auto upper = [&](const fde_operator* o, double& hi, double& lo) -> hodlr_status {
    std::vector<double> dp(o->n), dm(o->n);
    HIP_TRY(hipMemcpy(dp.data(), o->d_plus, o->n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dm.data(), o->d_minus, o->n * sizeof(double), hipMemcpyDeviceToHost));
    double mx = 0.0, mxp = 0.0, mxm = 0.0;
    for (int64_t i = 0; i < o->n; ++i) {
      mx = std::max(mx, dp[i] + dm[i]);
      mxp = std::max(mxp, dp[i]);
      mxm = std::max(mxm, dm[i]);
    }
    const double nu = o->dt / std::pow(o->dx, o->alpha);
    if (o->discretization == FDE_FE) {
      const double p = 3.0 - o->alpha, ig = 1.0 / std::tgamma(4.0 - o->alpha);
      const double w1 = (std::pow(2.0, p) - 4.0) * ig;
      const double w2 = (std::pow(3.0, p) - 4.0 * std::pow(2.0, p) + 6.0) * ig;
      const double sumabs = -2.0 * (w1 + std::min(w2, 0.0));
      hi = o->shift + 3.0 * nu * (mxp + mxm) * sumabs;
      lo = o->shift * (2.0 / 3.0) + nu * (-w1) * mx;   // the largest diagonal entry
      return HODLR_OK;
    }
    hi = o->shift + 2.0 * nu * o->alpha * mx;
    lo = o->shift + nu * o->alpha * mx;       // the largest diagonal entry: <= the 2-norm
    return HODLR_OK;
  };
  double b1 = 0, b2 = 0, l1 = 0, l2 = 0;
  hodlr_status st = upper(opx, b1, l1);
  if (st == HODLR_OK) st = upper(opy, b2, l2);
  if (st != HODLR_OK) { fde2d_plan_destroy(P); return st; }
  const double a1 = opx->shift, a2 = opy->shift;
  P->iv[0] = a1;
  P->iv[1] = b1;
  P->iv[2] = a2;
  P->iv[3] = b2;
  P->bound_x = l1;
  P->bound_y = l2;
  if (opx->discretization == FDE_FE) { P->fe = true; P->mass_x = 2.0 / 3.0; P->mc_x = 0.25; }
  if (opy->discretization == FDE_FE) { P->fe = true; P->mass_y = 2.0 / 3.0; P->mc_y = 0.25; }
  int J = 1;
  for (; J <= opts->max_shifts; ++J) {
    zolotarev_shifts(a1, b1, a2, b2, J, P->p, P->q);
    if (zolotarev_bound(a1, b1, a2, b2, P->p, P->q) <= 0.1 * opts->tol) break;
  }
  J = std::min(J, opts->max_shifts);
  zolotarev_shifts(a1, b1, a2, b2, J, P->p, P->q);
  P->J = J;
  // Shift pairs are applied in an interleaved order (the two ends of the
  // sorted list, then midpoints breadth first), so that every prefix of the
  // sweep spreads over both spectral intervals: the sweep can stop as soon as
  // the residual meets the target, which a first guess with a small residual
  // reaches early.
  {
    std::vector<int> ord;
    std::vector<char> used(J, 0);
    auto take = [&](int i) {
      if (i >= 0 && i < J && !used[i]) {
        used[i] = 1;
        ord.push_back(i);
      }
    };
    take(0);
    take(J - 1);
    std::vector<std::pair<int, int>> seg{{0, J - 1}};
    while (!seg.empty()) {
      std::vector<std::pair<int, int>> next;
      for (auto [lo, hi] : seg) {
        if (hi - lo < 2) continue;
        const int mid = (lo + hi) / 2;
        take(mid);
        next.push_back({lo, mid});
        next.push_back({mid, hi});
      }
      seg.swap(next);
    }
    for (int i = 0; i < J; ++i) take(i);
    P->order = ord;
  }
  // batched shifted operator: x items shift_x + q_j, y items shift_y + p_j
  std::vector<fde_operator> ops;
  for (int j = 0; j < J; ++j) { fde_operator o = *opx; o.shift = opx->shift + P->q[j]; ops.push_back(o); }
  for (int j = 0; j < J; ++j) { fde_operator o = *opy; o.shift = opy->shift + P->p[j]; ops.push_back(o); }
  hodlr_opts ho = *hopts;
  ho.refine_max = 0;
  fde_operator ex[2] = {*opx, *opy};
  size_t need_mat = 0, need_ex = 0;
  if (sizing || ws) {
    st = hodlr_workspace_size(ops.data(), int(ops.size()), &ho, &need_mat);
    if (st == HODLR_OK) st = hodlr_workspace_size(ex, 2, &ho, &need_ex);
    if (st != HODLR_OK) { fde2d_plan_destroy(P); return st; }
    need_mat = (need_mat + 255) & ~size_t(255);
    need_ex = (need_ex + 255) & ~size_t(255);
  }
  int64_t total_rows = 0;
  std::vector<WorkUnit> pw;
  std::vector<NodeUnit> pn;
  if (!sizing) {
    char* wsc = static_cast<char*>(ws);
    if (ws && ws_bytes < need_mat + need_ex) { fde2d_plan_destroy(P); return set_arg(ctx, 7); }
    st = ws ? hodlr_build_ws(ctx, ops.data(), int(ops.size()), &ho, wsc, need_mat, &P->mat)
            : hodlr_build(ctx, ops.data(), int(ops.size()), &ho, &P->mat);
    if (st != HODLR_OK) { fde2d_plan_destroy(P); return st; }
    hodlr_info fi{};
    st = hodlr_factor(ctx, P->mat, &fi);
    if (st != HODLR_OK && st != HODLR_ERANK) { fde2d_plan_destroy(P); return st; }
    st = ws ? hodlr_build_ws(ctx, ex, 2, &ho, wsc + need_mat, need_ex, &P->exact)
            : hodlr_build(ctx, ex, 2, &ho, &P->exact);
    if (st != HODLR_OK) { fde2d_plan_destroy(P); return st; }
    if (ws) {
      P->ws = wsc + need_mat + need_ex;
      P->ws_bytes = ws_bytes - need_mat - need_ex;
    }
    // per-pair solve unit lists (x_j leaves/nodes, then y_j)
    hodlr_mat m = P->mat;
    total_rows = m->total_n;
    std::vector<int> wo(m->batch + 1, 0), no(m->batch + 1, 0);
    for (const WorkUnit& w : m->wu_h) wo[w.item + 1]++;
    for (const NodeUnit& u : m->nu_h) no[u.item + 1]++;
    for (int i = 0; i < m->batch; ++i) { wo[i + 1] += wo[i]; no[i + 1] += no[i]; }
    for (int j = 0; j < J; ++j) {
      P->pwu_off.push_back(int(pw.size()));
      P->pnu_off.push_back(int(pn.size()));
      for (int it : {j, J + j}) {
        pw.insert(pw.end(), m->wu_h.begin() + wo[it], m->wu_h.begin() + wo[it + 1]);
        pn.insert(pn.end(), m->nu_h.begin() + no[it], m->nu_h.begin() + no[it + 1]);
      }
      P->pwu_cnt.push_back(int(pw.size()) - P->pwu_off.back());
      P->pnu_cnt.push_back(int(pn.size()) - P->pnu_off.back());
    }
  } else {
    // the unit lists hold one entry per leaf and internal node of every shifted problem
    int64_t leaves = 0, nodes = 0;
    for (const fde_operator& o : ops) {
      const int L = levels_for(o.n, ho.leaf);
      leaves += int64_t(1) << L;
      nodes += (int64_t(1) << L) - 1;
      total_rows += o.n;
    }
    pw.resize(size_t(leaves));
    pn.resize(size_t(nodes));
  }
  const int64_t nx = P->nx, ny = P->ny;
  const int64_t mr = std::max(nx, ny);
  P->cap_gram = int(2 * ((mr + kLrRows - 1) / kLrRows));
  P->slot_units = P->cap_gram + 2 + int(2 * ((mr + 255) / 256));
  bool ok = plan_alloc(P, &P->pair_wu, pw.size()) == HODLR_OK && plan_alloc(P, &P->pair_nu, pn.size()) == HODLR_OK &&
            plan_alloc(P, &P->G, nx * kMaxCat) == HODLR_OK && plan_alloc(P, &P->H, ny * kMaxCat) == HODLR_OK &&
            plan_alloc(P, &P->G0, nx * kMaxCat) == HODLR_OK && plan_alloc(P, &P->H0, ny * kMaxCat) == HODLR_OK &&
            plan_alloc(P, &P->R1, nx * kMaxCat) == HODLR_OK && plan_alloc(P, &P->R1w, ny * kMaxCat) == HODLR_OK &&
            plan_alloc(P, &P->xin, total_rows * kMaxCat) == HODLR_OK &&
            plan_alloc(P, &P->ex_in, (nx + ny) * kMaxCat) == HODLR_OK &&
            plan_alloc(P, &P->ex_out, (nx + ny) * kMaxCat) == HODLR_OK && plan_alloc(P, &P->ranks, kR_N) == HODLR_OK &&
            plan_alloc(P, &P->units, kLrSlots * P->slot_units) == HODLR_OK &&
            plan_alloc(P, &P->gpart, kLrSlots * P->cap_gram * kG2) == HODLR_OK &&
            plan_alloc(P, &P->grams, 2 * kLrSlots * kG2) == HODLR_OK &&
            plan_alloc(P, &P->mbuf, kLrSlots * 2 * kMaxCat * kRS) == HODLR_OK &&
            plan_alloc(P, &P->frob, kLrSlots) == HODLR_OK;
  ok = ok && plan_alloc(P, &P->counters, 1) == HODLR_OK && plan_alloc(P, &P->lrs_cpart, ((std::max(nx, ny) + kLrsSlice - 1) / kLrsSlice) * kLrsCols * kLrsK) == HODLR_OK &&
       plan_alloc(P, &P->lrs_t, kLrsCols * kLrsK) == HODLR_OK &&
       plan_alloc(P, &P->lrs_part, ((nx + 63) / 64) * ((ny + 63) / 64)) == HODLR_OK &&
       plan_alloc(P, &P->dnorm, 1) == HODLR_OK && plan_alloc(P, &P->om, ny * kSketch) == HODLR_OK &&
       plan_alloc(P, &P->sk_y, nx * kSketch) == HODLR_OK && plan_alloc(P, &P->sk_q1, nx * kSketch) == HODLR_OK &&
       plan_alloc(P, &P->sk_q2, nx * kSketch) == HODLR_OK && plan_alloc(P, &P->sk_b, ny * kSketch) == HODLR_OK &&
       plan_alloc(P, &P->eye, kSketch * kSketch) == HODLR_OK &&
       plan_alloc(P, &P->sk_junk, kSketch * kSketch) == HODLR_OK;
  if (P->fe)
    ok = ok && plan_alloc(P, &P->cz, nx * (kMaxCat + kRS)) == HODLR_OK &&
         plan_alloc(P, &P->cw, ny * (kMaxCat + kRS)) == HODLR_OK &&
         plan_alloc(P, &P->ex_mass, (nx + ny) * kMaxCat) == HODLR_OK;
  for (int k = 0; k < 2 && ok; ++k)
    ok = plan_alloc(P, &P->Zc[k], nx * kRS) == HODLR_OK && plan_alloc(P, &P->Wc[k], ny * kRS) == HODLR_OK &&
         plan_alloc(P, &P->Zx[k], nx * kRS) == HODLR_OK && plan_alloc(P, &P->Wx[k], ny * kRS) == HODLR_OK &&
         plan_alloc(P, &P->Zd[k], nx * kRS) == HODLR_OK && plan_alloc(P, &P->Wd[k], ny * kRS) == HODLR_OK &&
         plan_alloc(P, &P->Ze[k], nx * kRS) == HODLR_OK && plan_alloc(P, &P->We[k], ny * kRS) == HODLR_OK;
  if (!ok) {
    fde2d_plan_destroy(P);
    return ws ? set_arg(ctx, 7) : HODLR_ENOMEM;
  }
  if (sizing) {
    *need = need_mat + need_ex + P->ws_used + 256;   // + alignment of the workspace's own start
    fde2d_plan_destroy(P);
    return HODLR_OK;
  }
  if (hipMemcpy(P->pair_wu, pw.data(), pw.size() * sizeof(WorkUnit), hipMemcpyHostToDevice) != hipSuccess ||
      (!pn.empty() && hipMemcpy(P->pair_nu, pn.data(), pn.size() * sizeof(NodeUnit), hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemsetAsync(P->ranks, 0, kR_N * sizeof(int32_t), s) != hipSuccess ||
      hipMemsetAsync(P->counters, 0, sizeof(double), s) != hipSuccess) {
    fde2d_plan_destroy(P);
    return HODLR_EHIP;
  }
  static bool attr = false;
  if (!attr) {
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lr_core), hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(kFactorLdsBytes)));
    attr = true;
  }
  HIP_TRY(hipStreamSynchronize(s));
  *out = P;
  return HODLR_OK;
}

hodlr_status fde2d_plan_create(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                               const hodlr_opts* hopts, const fde2d_opts* opts, fde2d_plan* out) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  return plan2d_impl(ctx, opx, opy, hopts, opts, nullptr, 0, out, nullptr);
}

hodlr_status fde2d_plan_counters(fde2d_plan P, double* values, int count, int reset) {
  if (!P || !values || count < 0) return HODLR_EINVAL;
  double core = 0.0;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(&core, P->counters, sizeof(double), hipMemcpyDeviceToHost));
  hodlr_mat_info mi{};
  if (P->mat) TRY(hodlr_get_info(P->mat, &mi));
  const double v[7] = {core, P->lrs_flops, double(mi.bytes_factors), double(P->J), double(mi.max_rank_factors),
                       double(P->ek_J), P->ek_gemm_flops};
  for (int i = 0; i < count && i < 7; ++i) values[i] = v[i];
  if (reset) {
    HIP_TRY(hipMemset(P->counters, 0, sizeof(double)));
    P->lrs_flops = 0.0;
    P->ek_gemm_flops = 0.0;
  }
  return HODLR_OK;
}

hodlr_status fde2d_plan_workspace_size(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                                       const hodlr_opts* hopts, const fde2d_opts* opts, size_t* bytes) {
  if (!ctx) return HODLR_EINVAL;
  if (!bytes) return set_arg(ctx, 6);
  size_t need = 0;
  const hodlr_status st = plan2d_impl(ctx, opx, opy, hopts, opts, nullptr, 0, nullptr, &need);
  if (st != HODLR_OK) return st;
  *bytes = need;
  return HODLR_OK;
}

hodlr_status fde2d_plan_create_ws(hodlr_ctx ctx, const fde_operator* opx, const fde_operator* opy,
                                  const hodlr_opts* hopts, const fde2d_opts* opts, void* workspace,
                                  size_t ws_bytes, fde2d_plan* out) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!workspace) return set_arg(ctx, 6);
  if (!out) return set_arg(ctx, 8);
  size_t need = 0;
  const hodlr_status st = plan2d_impl(ctx, opx, opy, hopts, opts, nullptr, 0, nullptr, &need);
  if (st != HODLR_OK) return st;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(workspace);
  const uintptr_t a1 = (a0 + 255) & ~uintptr_t(255);
  if (ws_bytes < need || ws_bytes < (a1 - a0)) return set_arg(ctx, 7);
  return plan2d_impl(ctx, opx, opy, hopts, opts, reinterpret_cast<void*>(a1), ws_bytes - (a1 - a0), out, nullptr);
}

hodlr_status fde2d_sylvester_step_guess(hodlr_ctx ctx, fde2d_plan P, const lr_matrix* U_m, const lr_matrix* F,
                                        double dt, const lr_matrix* X0, lr_matrix* U_next, hodlr_info* info) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!P) return set_arg(ctx, 2);
  if (!U_m || U_m->rank < 0 || U_m->rank > kMaxCat || (U_m->rank > 0 && (!U_m->Z || !U_m->W))) return set_arg(ctx, 3);
  if (!F || F->rank < 0 || F->rank > kRS || (F->rank > 0 && (!F->Z || !F->W))) return set_arg(ctx, 4);
  if (X0 && (X0->rank < 0 || X0->rank > kMaxCat || (X0->rank > 0 && (!X0->Z || !X0->W))))
    return set_arg(ctx, 6);
  if (!U_next || !U_next->Z || !U_next->W || U_next->capacity < 1) return set_arg(ctx, 7);
  hipStream_t s = ctx->stream;
  const int64_t nx = P->nx, ny = P->ny;
  const double tol = P->opts.tol;
  int32_t hr[kR_N];
  lr_matrix um_e{}, f_e{};
  if (P->fe) {
    // Finite elements: C = E_x (U_m + dt F) E_y, so the caller's factors
    // enter with the mass matrices applied (exact: E is tridiagonal).
    mass_cols(nx, U_m->rank, P->mass_x, P->mc_x, U_m->Z, U_m->ldz, P->cz, nx, 1.0, s);
    mass_cols(ny, U_m->rank, P->mass_y, P->mc_y, U_m->W, U_m->ldw, P->cw, ny, 1.0, s);
    mass_cols(nx, F->rank, P->mass_x, P->mc_x, F->Z, F->ldz, P->cz + kMaxCat * nx, nx, 1.0, s);
    mass_cols(ny, F->rank, P->mass_y, P->mc_y, F->W, F->ldw, P->cw + kMaxCat * ny, ny, 1.0, s);
    um_e = lr_matrix{nx, U_m->rank, U_m->rank, nx, ny, P->cz, P->cw};
    f_e = lr_matrix{nx, F->rank, F->rank, nx, ny, P->cz + kMaxCat * nx, P->cw + kMaxCat * ny};
    U_m = &um_e;
    F = &f_e;
  }
  HIP_TRY(hipMemsetAsync(P->ranks + kR_CAP, 0, sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P->ranks + kR_X0, 0, 2 * sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(P->ranks + kR_K0, 0, 2 * sizeof(int32_t), s));
  // Right-hand side of the first sweep: C = [Z_m, dt F_Z][W_m, F_W]^T
  // recompressed into G0, H0 (a factor U_m wider than kRS first on its own).
  // The exact C, for the residuals, is the caller's factors themselves.
  {
    const lr_matrix* um = U_m;
    lr_matrix pre{};
    if (U_m->rank > kRS || U_m->rank + F->rank > kMaxCat) {
      LrJob pj{};
      pj.X.g[0] = grp(U_m->Z, U_m->ldz, nullptr, U_m->rank, 1.0);
      pj.X.g[1] = pj.X.g[2] = grp_none();
      pj.Y.g[0] = grp(U_m->W, U_m->ldw, nullptr, U_m->rank, 1.0);
      pj.Y.g[1] = pj.Y.g[2] = grp_none();
      pj.rows_x = nx;
      pj.rows_y = ny;
      pj.rank_out = P->ranks + kR_T;
      pj.tau = 0.0;
      pj.tau_rel = 1e-3 * tol;
      pj.rmax = kRS;
      pj.U = P->R1;
      pj.ldu = nx;
      pj.V = P->R1w;
      pj.ldv = ny;
      TRY(run_lr(P, pj, 0, true, s));
      TRY(read_ranks(P, hr, s));
      pre.rows = nx;
      pre.rank = hr[kR_T];
      pre.ldz = nx;
      pre.ldw = ny;
      pre.Z = P->R1;
      pre.W = P->R1w;
      um = &pre;
    }
    LrJob cj{};
    cj.X.g[0] = grp(um->Z, um->ldz, nullptr, um->rank, 1.0);
    cj.X.g[1] = grp(F->Z, F->ldz, nullptr, F->rank, dt);
    cj.X.g[2] = grp_none();
    cj.Y.g[0] = grp(um->W, um->ldw, nullptr, um->rank, 1.0);
    cj.Y.g[1] = grp(F->W, F->ldw, nullptr, F->rank, 1.0);
    cj.Y.g[2] = grp_none();
    cj.rows_x = nx;
    cj.rows_y = ny;
    cj.rank_out = P->ranks + kR_C;
    cj.tau = 0.0;
    cj.tau_rel = 1e-3 * tol;
    cj.rmax = kRS;
    cj.U = P->G0;
    cj.ldu = nx;
    cj.V = P->H0;
    cj.ldv = ny;
    if (um->rank + F->rank > 0) {
      TRY(run_lr(P, cj, 0, true, s));
    } else {
      HIP_TRY(hipMemsetAsync(P->ranks + kR_C, 0, sizeof(int32_t), s));
    }
  }
  TRY(read_ranks(P, hr, s));
  const int rc = hr[kR_C];
  // ||C||_F, formed entry by entry from the caller's factors
  LrSum csum{};
  csum.nx = nx;
  csum.ny = ny;
  csum.g[csum.ng++] = LrsGroup{U_m->Z, U_m->ldz, U_m->W, U_m->ldw, nullptr, U_m->rank, 1.0};
  csum.g[csum.ng++] = LrsGroup{F->Z, F->ldz, F->W, F->ldw, nullptr, F->rank, dt};
  double cnorm = 0.0;
  TRY(dense_norm(P, csum, cnorm, s));
  // The solution is kept as two low-rank terms: X = X_main + X_corr.  X_main
  // (Zx/Wx, rank at kR_X0 + parity) is the first sweep's result, or the
  // caller's guess; X_corr (Zc/Wc, kR_K0 + parity) sums the corrections.  A
  // recompression of a sum resolves its terms only to about sqrt(u) times its
  // norm, so the corrections, each a small fraction of X, are summed apart
  // from X_main; the residual C - A X - X B^T of the sum is formed entry by
  // entry (dense_norm), which resolves it to about u times its terms.
  int xpar = 0, kpar = 0, total_steps = 0, sweeps = 0;
  const bool verbose = getenv("HODLR_VERBOSE") != nullptr;
  double rel_res = 1.0, rel_corr = 0.0, eta = 1.0, guess_res = 0.0;
  bool warm = false, fallback = false;
  // R = C - A X - X B^T for X = X_main + X_corr: its norm relative to
  // ||C||_F, and the normwise backward error eta (||A||_2, ||B||_2 replaced by
  // lower bounds, so eta is an upper bound of the true one).
  LrSum rsum{};
  double xnorm = 0.0;
  auto residual = [&](double& rel) -> hodlr_status {
    TRY(read_ranks(P, hr, s));
    const int rx = hr[kR_X0 + xpar], rk = hr[kR_K0 + kpar];
    const int64_t ld = nx + ny;
    copy_cols(nx, nullptr, rx, P->Zx[xpar], nx, P->ex_in, ld, 1.0, s);
    copy_cols(ny, nullptr, rx, P->Wx[xpar], ny, P->ex_in + nx, ld, 1.0, s);
    if (rk > 0) {
      copy_cols(nx, nullptr, rk, P->Zc[kpar], nx, P->ex_in + rx * ld, ld, 1.0, s);
      copy_cols(ny, nullptr, rk, P->Wc[kpar], ny, P->ex_in + rx * ld + nx, ld, 1.0, s);
    }
    if (rx + rk > 0) launch_fft_matvec(P->exact, P->ex_in, ld, P->ex_out, ld, nullptr, 0, rx + rk, s);
    LrSum& r = rsum;
    r = csum;
    if (!P->fe) {
      r.g[r.ng++] = LrsGroup{P->ex_out, ld, P->Wx[xpar], ny, nullptr, rx, -1.0};             // A Z_main W_main^T
      r.g[r.ng++] = LrsGroup{P->Zx[xpar], nx, P->ex_out + nx, ld, nullptr, rx, -1.0};        // Z_main (B W_main)^T
      r.g[r.ng++] = LrsGroup{P->ex_out + rx * ld, ld, P->Wc[kpar], ny, nullptr, rk, -1.0};   // A Z_corr W_corr^T
      r.g[r.ng++] = LrsGroup{P->Zc[kpar], nx, P->ex_out + rx * ld + nx, ld, nullptr, rk, -1.0};
    } else {
      // A X E_y + E_x X B^T: (A Z)(E_y W)^T + (E_x Z)(B W)^T for both terms
      mass_cols(nx, rx + rk, P->mass_x, P->mc_x, P->ex_in, ld, P->ex_mass, ld, 1.0, s);
      mass_cols(ny, rx + rk, P->mass_y, P->mc_y, P->ex_in + nx, ld, P->ex_mass + nx, ld, 1.0, s);
      for (int t = 0; t < 2; ++t) {
        const int64_t c0 = t == 0 ? 0 : rx * ld;
        const int rc_t = t == 0 ? rx : rk;
        r.g[r.ng++] = LrsGroup{P->ex_out + c0, ld, P->ex_mass + c0 + nx, ld, nullptr, rc_t, -1.0};
        r.g[r.ng++] = LrsGroup{P->ex_mass + c0, ld, P->ex_out + c0 + nx, ld, nullptr, rc_t, -1.0};
      }
    }
    double rn = 0.0;
    TRY(dense_norm(P, r, rn, s));
    // ||X||_F of the main term (Gram trace): the correction term is a small
    // fraction of it
    double x2 = 0.0;
    if (rx > 0) {
      LrJob xj{};
      xj.X.g[0] = grp(P->Zx[xpar], nx, P->ranks + kR_X0 + xpar, 0, 1.0);
      xj.X.g[1] = xj.X.g[2] = grp_none();
      xj.Y.g[0] = grp(P->Wx[xpar], ny, P->ranks + kR_X0 + xpar, 0, 1.0);
      xj.Y.g[1] = xj.Y.g[2] = grp_none();
      xj.rows_x = nx;
      xj.rows_y = ny;
      TRY(run_lr(P, xj, 6, false, s));
      TRY(read_frob(P, 6, &x2, s));
    }
    xnorm = std::sqrt(std::max(x2, 0.0));
    rel = cnorm > 0 ? rn / cnorm : 0.0;
    // ||A X E_y + E_x X B^T|| <= (||A|| ||E_y|| + ||E_x|| ||B||) ||X||; the
    // masses' lower bounds are their diagonals (1 for the identity)
    const double scale = (P->bound_x * P->mass_y + P->mass_x * P->bound_y) * xnorm + cnorm;
    eta = scale > 0 ? rn / scale : 0.0;
    return HODLR_OK;
  };
  // the next right-hand side G H^T: R compressed (rank at kR_R0)
  auto residual_rhs = [&]() -> hodlr_status {
    return compress_lrsum(P, rsum, 1e-6, 0x5eedULL + uint64_t(total_steps), kRS, P->G, nx, P->H, ny,
                          P->ranks + kR_R0, s);
  };
  if (X0 && X0->rank > 0 && rc > 0) {
    // first guess: X_main = X0 (recompressed if wider than kRS); the first
    // sweep solves for its residual
    if (X0->rank <= kRS) {
      copy_cols(nx, nullptr, X0->rank, X0->Z, X0->ldz, P->Zx[0], nx, 1.0, s);
      copy_cols(ny, nullptr, X0->rank, X0->W, X0->ldw, P->Wx[0], ny, 1.0, s);
      const int32_t rk = X0->rank;
      HIP_TRY(hipMemcpyAsync(P->ranks + kR_X0, &rk, sizeof(int32_t), hipMemcpyHostToDevice, s));
    } else {
      LrJob gj{};
      gj.X.g[0] = grp(X0->Z, X0->ldz, nullptr, X0->rank, 1.0);
      gj.X.g[1] = gj.X.g[2] = grp_none();
      gj.Y.g[0] = grp(X0->W, X0->ldw, nullptr, X0->rank, 1.0);
      gj.Y.g[1] = gj.Y.g[2] = grp_none();
      gj.rows_x = nx;
      gj.rows_y = ny;
      gj.rank_out = P->ranks + kR_X0;
      gj.tau = 0.0;
      gj.tau_rel = 0.1 * tol;
      gj.rmax = kRS;
      gj.U = P->Zx[0];
      gj.ldu = nx;
      gj.V = P->Wx[0];
      gj.ldv = ny;
      TRY(run_lr(P, gj, 4, true, s));
    }
    double rel0 = 0.0;
    TRY(residual(rel0));
    guess_res = rel0;
    // The J shifts reduce a residual by about 0.1 tol, i.e. by
    // (0.1 tol)^(1/J) per shift.  The guess is worth taking only if its
    // residual saves at least one block of four shifts (the sweep tests for
    // convergence every four).  Otherwise the plain step runs, so a guess
    // never costs ADI steps.
    const double accept = std::pow(0.1 * tol, 4.0 / std::max(P->J, 4));
    if (rel0 <= accept) {
      warm = true;
      rel_res = rel0;
    } else {
      fallback = true;          // the guess is no better than zero: plain solve
      HIP_TRY(hipMemsetAsync(P->ranks + kR_X0, 0, sizeof(int32_t), s));
    }
  }
  hodlr_status res = HODLR_OK;
  if (rc > 0) {
    if (!warm) {
      // sweep 0 on C itself: its result is X_main
      copy_cols(nx, P->ranks + kR_C, 0, P->G0, nx, P->G, nx, 1.0, s);
      copy_cols(ny, P->ranks + kR_C, 0, P->H0, ny, P->H, ny, 1.0, s);
      HIP_TRY(hipMemcpyAsync(P->ranks + kR_R0, P->ranks + kR_C, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      // With reduced-precision factors each shifted solve carries errors of
      // about the factors' precision, which the first sweep cannot go below:
      // it stops there, and the corrections (whose residuals are exact) take
      // the solution the rest of the way.
      // The sweeps aim one decade below the tolerance (relative to ||C||).
      const int fp = P->mat->opts.prec;
      const double first = fp == HODLR_FP64 ? 0.1 * tol : std::max(0.1 * tol, fp == HODLR_MIXED_FP32 ? 1e-6 : 1e-3);
      int steps = 0, dpar = 0;
      TRY(step_solve(P, rc, first * std::max(cnorm, 1e-300), 0, steps, dpar, s));
      total_steps += steps;
      LrJob mj{};
      mj.X.g[0] = grp(P->Zd[dpar], nx, P->ranks + kR_D0 + dpar, 0, 1.0);
      mj.X.g[1] = mj.X.g[2] = grp_none();
      mj.Y.g[0] = grp(P->Wd[dpar], ny, P->ranks + kR_D0 + dpar, 0, 1.0);
      mj.Y.g[1] = mj.Y.g[2] = grp_none();
      mj.rows_x = nx;
      mj.rows_y = ny;
      mj.rank_out = P->ranks + kR_X0;
      mj.tau = 0.0;
      mj.tau_rel = 0.1 * tol;
      mj.rmax = P->opts.max_rank;
      mj.U = P->Zx[0];
      mj.ldu = nx;
      mj.V = P->Wx[0];
      mj.ldv = ny;
      TRY(run_lr(P, mj, 4, true, s));
      TRY(residual(rel_res));
      if (verbose)
        fprintf(stderr, "hodlr_fde: 2D step: first sweep: %d ADI steps, backward error %.2e, |R|/|C| %.2e\n",
                steps, eta, rel_res);
    }
    // corrections: A D + D B^T = R, X_corr <- X_corr + D, while the normwise
    // backward error ||R|| / ((||A|| + ||B||) ||X|| + ||C||) exceeds tol, and
    // with reduced-precision factors also while the forward error estimate
    // of iterative refinement exceeds tol: corrections shrink geometrically,
    // so the error left after D_k is about |D_k| |D_k| / |D_{k-1}| (D_0 = X).
    // The backward error weighs the residual by ||A|| + ||B||, so errors in
    // the smooth modes, where A and B are small, can hide below it, and the
    // low-precision solves leave errors in every mode.  With BF16 factors the
    // error of a shifted solve, about u_bf16 kappa(A + q E), nears 1 for the
    // small shifts: the late corrections shrink by only 0.3-0.5 each and not
    // steadily, so the ratio undershoots; there the estimate is |D_k| itself.
    const bool mixed = P->mat->opts.prec != HODLR_FP64;
    const bool slow = P->mat->opts.prec == HODLR_MIXED_BF16;
    double fwd_est = mixed ? HUGE_VAL : 0.0, prev_corr = 1.0;
    for (sweeps = 0; sweeps < kMaxCorrections && (eta > tol || fwd_est > tol); ++sweeps) {
      TRY(residual_rhs());
      TRY(read_ranks(P, hr, s));
      const int r0 = hr[kR_R0];
      if (r0 == 0) break;
      int steps = 0, dpar = 0;
      TRY(step_solve(P, r0, 0.1 * tol * std::max(cnorm, 1e-300), 1, steps, dpar, s));
      total_steps += steps;
      // ||D||_F (Gram trace), the size of the correction
      double d2 = 0.0;
      {
        LrJob nj{};
        nj.X.g[0] = grp(P->Zd[dpar], nx, P->ranks + kR_D0 + dpar, 0, 1.0);
        nj.X.g[1] = nj.X.g[2] = grp_none();
        nj.Y.g[0] = grp(P->Wd[dpar], ny, P->ranks + kR_D0 + dpar, 0, 1.0);
        nj.Y.g[1] = nj.Y.g[2] = grp_none();
        nj.rows_x = nx;
        nj.rows_y = ny;
        TRY(run_lr(P, nj, 5, false, s));
        TRY(read_frob(P, 5, &d2, s));
      }
      rel_corr = xnorm > 0 ? std::sqrt(std::max(d2, 0.0)) / xnorm : 0.0;
      if (mixed)
        fwd_est = slow ? rel_corr : rel_corr * std::min(1.0, rel_corr / std::max(prev_corr, 1e-300));
      prev_corr = rel_corr;
      // X_corr <- recompress([X_corr, D]).  An error e in X changes the
      // residual by up to (||A|| ||E_y|| + ||E_x|| ||B||) e, so the truncation
      // is absolute, at 0.1 tol of the backward error's scale over that norm
      LrJob kj{};
      kj.X.g[0] = grp(P->Zc[kpar], nx, P->ranks + kR_K0 + kpar, 0, 1.0);
      kj.X.g[1] = grp(P->Zd[dpar], nx, P->ranks + kR_D0 + dpar, 0, 1.0);
      kj.X.g[2] = grp_none();
      kj.Y.g[0] = grp(P->Wc[kpar], ny, P->ranks + kR_K0 + kpar, 0, 1.0);
      kj.Y.g[1] = grp(P->Wd[dpar], ny, P->ranks + kR_D0 + dpar, 0, 1.0);
      kj.Y.g[2] = grp_none();
      kj.rows_x = nx;
      kj.rows_y = ny;
      kj.rank_out = P->ranks + kR_K0 + (1 - kpar);
      const double lnorm = P->bound_x * P->mass_y + P->mass_x * P->bound_y;
      kj.tau = 0.1 * tol * (lnorm * xnorm + cnorm) / lnorm;
      kj.tau_rel = 0.0;
      kj.rmax = kRS;
      kj.capped = P->ranks + kR_CAP;
      kj.U = P->Zc[1 - kpar];
      kj.ldu = nx;
      kj.V = P->Wc[1 - kpar];
      kj.ldv = ny;
      TRY(run_lr(P, kj, 7, true, s));
      kpar = 1 - kpar;
      TRY(residual(rel_res));
      if (verbose)
        fprintf(stderr, "hodlr_fde: 2D step: correction %d: %d ADI steps, |D|/|X| %.2e, forward error estimate "
                "%.2e, backward error %.2e, |R|/|C| %.2e\n", sweeps + 1, steps, rel_corr, fwd_est, eta, rel_res);
    }
    if (eta > tol || fwd_est > tol) res = HODLR_ENOCONV;
  } else {
    rel_res = 0.0;
    eta = 0.0;
  }
  TRY(read_ranks(P, hr, s));
  const int rx = hr[kR_X0 + xpar], rk = hr[kR_K0 + kpar];
  if (rx + rk > U_next->capacity) return set_arg(ctx, 7);
  copy_cols(nx, nullptr, rx, P->Zx[xpar], nx, U_next->Z, U_next->ldz, 1.0, s);
  copy_cols(ny, nullptr, rx, P->Wx[xpar], ny, U_next->W, U_next->ldw, 1.0, s);
  if (rk > 0) {
    copy_cols(nx, nullptr, rk, P->Zc[kpar], nx, U_next->Z + rx * U_next->ldz, U_next->ldz, 1.0, s);
    copy_cols(ny, nullptr, rk, P->Wc[kpar], ny, U_next->W + rx * U_next->ldw, U_next->ldw, 1.0, s);
  }
  U_next->rank = rx + rk;
  if (hr[kR_CAP] && res == HODLR_OK) res = HODLR_ERANK;
  if (hr[kR_CAP] && verbose)
    fprintf(stderr, "hodlr_fde: 2D step: rank cap reached in work slots 0x%x\n", unsigned(hr[kR_CAP]));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = res;
    info->refine_iters = total_steps;
    info->rel_residual = rel_res;
    info->rel_correction = rel_corr;
    info->backward_error = eta;
    info->guess_residual = guess_res;
    info->max_rank = rx + rk;
    info->leaf = -1;
    info->row = -1;
    info->used_fallback = fallback ? 1 : 0;
  }
  return res;
}

hodlr_status fde2d_field_from_lr(hodlr_ctx ctx, fde2d_plan P, const lr_matrix* X, float* out) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!P) return set_arg(ctx, 2);
  if (!X || X->rank < 0 || (X->rank > 0 && (!X->Z || !X->W))) return set_arg(ctx, 3);
  if (!out) return set_arg(ctx, 4);
  const int64_t tot = P->nx * P->ny;
  HFDE_LAUNCH(k_lr_to_dense, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, ctx->stream, P->nx, P->ny, X->rank, X->Z,
              X->ldz, X->W, X->ldw, out);
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status fde2d_compress_field(hodlr_ctx ctx, fde2d_plan P, const float* X, double tol, uint64_t seed,
                                  lr_matrix* out) {
  if (!ctx) return HODLR_EINVAL;
  TimerScope ts_(ctx);
  if (!P) return set_arg(ctx, 2);
  if (!X) return set_arg(ctx, 3);
  if (!(tol > 0.0)) return set_arg(ctx, 4);
  if (!out || !out->Z || !out->W || out->capacity < 1) return set_arg(ctx, 6);
  hipStream_t s = ctx->stream;
  TRY(compress_dense(P, X, tol, seed, std::min(out->capacity, P->opts.max_rank), out->Z, out->ldz, out->W, out->ldw,
                     P->ranks + kR_D1, s));
  int32_t hr[kR_N];
  TRY(read_ranks(P, hr, s));
  out->rank = hr[kR_D1];
  HIP_TRY(hipGetLastError());
  return HODLR_OK;
}

hodlr_status fde2d_sylvester_step(hodlr_ctx ctx, fde2d_plan P, const lr_matrix* U_m, const lr_matrix* F, double dt,
                                  lr_matrix* U_next, hodlr_info* info) {
  const hodlr_status st = fde2d_sylvester_step_guess(ctx, P, U_m, F, dt, nullptr, U_next, info);
  if (st == HODLR_EINVAL && ctx && ctx->last_arg == 7) ctx->last_arg = 6;
  return st;
}

hodlr_status fde2d_ek_workspace_size(hodlr_ctx ctx, fde2d_plan P, size_t* bytes) {
  if (!ctx) return HODLR_EINVAL;
  if (!P) return set_arg(ctx, 2);
  if (!bytes) return set_arg(ctx, 3);
  // count the solver's arrays as a sizing pass, on a copy of the plan's
  // fields (the plan's own pointers stay as they are)
  fde2d_plan_s scratch = *P;
  scratch.sizing = true;
  scratch.ws_used = 0;
  const hodlr_status st = ek_alloc(&scratch);
  *bytes = scratch.ws_used + 256;                 // + alignment of the workspace's own start
  scratch.allocs.clear();
  return st;
}

hodlr_status fde2d_ek_attach_workspace(hodlr_ctx ctx, fde2d_plan P, void* workspace, size_t ws_bytes) {
  if (!ctx) return HODLR_EINVAL;
  if (!P) return set_arg(ctx, 2);
  if (!P->ws || P->ek_ws) return HODLR_ESTATE;    // only a workspace plan, once
  if (!workspace) return set_arg(ctx, 3);
  size_t need = 0;
  TRY(fde2d_ek_workspace_size(ctx, P, &need));
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(workspace);
  const uintptr_t a1 = (a0 + 255) & ~uintptr_t(255);
  if (ws_bytes < need || ws_bytes < a1 - a0) return set_arg(ctx, 4);
  // the plan's own arrays keep their places; later allocations (the solver's)
  // are carved from this workspace
  P->ek_ws = reinterpret_cast<char*>(a1);
  P->ws = P->ek_ws;
  P->ws_bytes = ws_bytes - (a1 - a0);
  P->ws_used = 0;
  return HODLR_OK;
}

hodlr_status fde2d_sylvester_step_ek(hodlr_ctx ctx, fde2d_plan P, const lr_matrix* U_m, const lr_matrix* F,
                                     double dt, lr_matrix* U_next, hodlr_info* info) {
  if (!ctx) return HODLR_EINVAL;
  if (!P) return set_arg(ctx, 2);
  P->use_ek = true;
  const hodlr_status st = fde2d_sylvester_step_guess(ctx, P, U_m, F, dt, nullptr, U_next, info);
  P->use_ek = false;
  if (st == HODLR_EINVAL && ctx->last_arg == 7) ctx->last_arg = 6;
  return st;
}

}  // extern "C"
