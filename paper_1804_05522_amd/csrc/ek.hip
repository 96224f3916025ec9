// Kernels of the extended Krylov solver of the per-step Sylvester equation
// (Sec. 4.3): products of the tall basis blocks and of the small projected
// matrices, batched LU factorisations and inverses of the shifted projected
// matrices T + s I, and the projected fADI pair update.
//
// The projected equation T_A Y + Y T_B^T = G H^T (T_A = U^T A U, T_B =
// V^T B V, U and V the orthonormal extended Krylov bases) is small (at most
// kEkMax on a side) and dense; it is solved by factored ADI with the plan's
// shift pairs on explicit inverses of T_A + q_j I and T_B + p_j I.

constexpr int kEkMax = 640;      // basis columns per side (T_A, T_B at most kEkMax x kEkMax)
constexpr int kEkPanel = 16;     // panel width of the blocked LU
constexpr int kEkSk = 40;        // sketch columns of the projected solution's range
constexpr int kEkSplit = 32;     // largest split of an inner dimension (k_ek_gemm partials)
constexpr int kEkWG = 1024;      // threads of the LU work-groups

// C = alpha op(A) op(B) + beta C for column-major A, B, C; op(X) = X (t = 0)
// or X^T (t = 1); C is M x N (N clipped to *ndev when ndev is set, the grid
// sized for N), the inner dimension K.  Work-group (x, y, z)
// takes the 64 x 64 output tile (x, y) over the inner indices
// [z kchunk, min(K, (z + 1) kchunk)): with one split (gridDim.z == 1) it
// writes C, otherwise its partial tile into part + z M N (M x N, ld M), which
// k_ek_gemm_sum adds up.  256 threads, 4 x 4 outputs each; 16-deep slices of
// both operands staged in LDS, loaded along the contiguous index.
__global__ void __launch_bounds__(256) k_ek_gemm(int ta, int tb, int M, int N, const int32_t* ndev, int64_t K,
                                                 int64_t kchunk, double alpha, const double* A, int64_t lda,
                                                 const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                                                 double* part) {
  constexpr int kK = 16;
  __shared__ double As[kK][65];
  __shared__ double Bs[kK][65];
  if (ndev) N = min(N, *ndev);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (j0 >= N) return;
  const int64_t k0 = int64_t(blockIdx.z) * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  double acc[4][4] = {};
  // the next slice's operands are loaded into registers while the current
  // slice is multiplied from LDS
  double va[4], vb[4];
  auto fetch = [&](int64_t kk) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int e = threadIdx.x + 256 * l;
      int i, k;
      if (ta == 0) { i = e % 64; k = e / 64; } else { k = e % kK; i = e / kK; }
      const int64_t kg = kk + k;
      va[l] = (i0 + i < M && kg < k1) ? (ta == 0 ? A[(i0 + i) + kg * lda] : A[kg + int64_t(i0 + i) * lda]) : 0.0;
      int j, kb;
      if (tb == 0) { kb = e % kK; j = e / kK; } else { j = e % 64; kb = e / 64; }
      const int64_t kgb = kk + kb;
      vb[l] = (j0 + j < N && kgb < k1) ? (tb == 0 ? B[kgb + int64_t(j0 + j) * ldb] : B[(j0 + j) + kgb * ldb]) : 0.0;
    }
  };
  if (k0 < k1) fetch(k0);
  for (int64_t kk = k0; kk < k1; kk += kK) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int e = threadIdx.x + 256 * l;
      if (ta == 0) As[e / 64][e % 64] = va[l]; else As[e % kK][e / kK] = va[l];
      if (tb == 0) Bs[e % kK][e / kK] = vb[l]; else Bs[e / 64][e % 64] = vb[l];
    }
    __syncthreads();
    if (kk + kK < k1) fetch(kk + kK);
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[k][tx + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[k][ty + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
    __syncthreads();
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + tx + 16 * r, j = j0 + ty + 16 * c;
      if (i >= M || j >= N) continue;
      if (gridDim.z == 1) {
        double* cp = C + i + int64_t(j) * ldc;
        *cp = alpha * acc[r][c] + (beta == 0.0 ? 0.0 : beta * *cp);
      } else {
        part[int64_t(blockIdx.z) * M * N + i + int64_t(j) * M] = acc[r][c];   // N clipped: same layout as the sum's
      }
    }
}

// C = alpha sum_z part_z + beta C (M x N, N clipped to *ndev when set).
__global__ void k_ek_gemm_sum(int M, int N, const int32_t* ndev, int nsplit, const double* part, double alpha,
                              double beta, double* C, int64_t ldc) {
  if (ndev) N = min(N, *ndev);
  const int64_t tot = int64_t(M) * N;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[int64_t(z) * tot + e];
    double* cp = C + (e % M) + (e / M) * ldc;
    *cp = alpha * s + (beta == 0.0 ? 0.0 : beta * *cp);
  }
}

// LU factorisation with partial pivoting (P (T + s_b I) = L U, L unit lower)
// of the batch's matrices, one work-group per matrix b: T = TA (order mA) for
// b < J, else TB (order mB), both ld ldt; s_b = shift[b]; the factors
// overwrite out + b stride (ld ldo), the pivot rows go to piv + b kEkMax, and
// flag[b] = 1 marks an exactly zero pivot.  Right-looking and blocked: a
// panel of kEkPanel columns is factored in LDS; its row interchanges, composed
// into one gather and one scatter, are applied to the other columns; the block
// row of U is solved with the panel's unit lower triangle in registers (a
// thread per column) and kept in LDS; the trailing matrix takes the
// rank-kEkPanel update on the FP64 matrix cores.  m <= kEkMax.
__global__ void __launch_bounds__(kEkWG) k_ek_lu(int J, int mA, const double* TA, int mB, const double* TB,
                                                 int64_t ldt, const double* shift, double* out, int64_t ldo,
                                                 int64_t stride, int32_t* piv, int32_t* flag) {
  constexpr int kP = kEkPanel;
  constexpr int kW = kEkWG / 64;
  // the panel (rows j0 .. m - 1, ld m - j0), then the block row of U right of
  // it, transposed ((m - j0 - kP) x kP, ld m - j0 - kP + 1)
  __shared__ double Sm[(2 * kEkMax - kP) * kP + kP];
  __shared__ int s_pv[kP];                   // the panel's pivot rows
  __shared__ double red_v[kW];
  __shared__ int red_i[kW];
  __shared__ double prow[kP];                // the pivot row of the current step
  __shared__ int s_p;
  __shared__ int sw_row[2 * kP], sw_src[2 * kP];
  const int b = blockIdx.x;
  const int m = b < J ? mA : mB;
  const double* T = b < J ? TA : TB;
  double* A = out + int64_t(b) * stride;
  int32_t* pv = piv + int64_t(b) * kEkMax;
  const double sh = shift[b];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t e = threadIdx.x; e < int64_t(m) * m; e += kEkWG) {
    const int i = int(e % m), j = int(e / m);
    A[i + int64_t(j) * ldo] = T[i + int64_t(j) * ldt] + (i == j ? sh : 0.0);
  }
  if (threadIdx.x == 0) flag[b] = 0;
  __syncthreads();
  for (int j0 = 0; j0 < m; j0 += kP) {
    const int nb = min(kP, m - j0), j1 = j0 + nb, mr = m - j0;
    double* Pn = Sm;
    double* Us = Sm + mr * kP;
    for (int e = threadIdx.x; e < mr * nb; e += kEkWG) {
      const int i = e % mr, c = e / mr;
      Pn[i + c * mr] = A[(j0 + i) + int64_t(j0 + c) * ldo];
    }
    __syncthreads();
    // pivot steps, two barriers each.  Candidates (largest magnitude in the
    // step's column, ties to the lowest row) are reduced within each wave,
    // then by wave 0, which also stages the pivot row; then a thread per row
    // below the step forms its multiplier and updates its row (the thread of
    // the pivot's row also carries out the interchange with row jj) and offers
    // its entry of the next column as the next step's candidate.
    // the wave's largest candidate and, among equal ones, the lowest lane's
    // (lanes hold at most one row each, in increasing order, so that is the
    // lowest row); lanes past `width` do not take part
    auto wave_best = [&](double& best, int& bi, int width) {
      double mx = lane < width ? best : -1.0;
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
      const unsigned long long hit = __ballot(lane < width && best == mx);
      const int src = hit ? __ffsll((long long)hit) - 1 : 0;
      bi = __shfl(bi, src);
      best = hit ? mx : best;
      best = __shfl(best, src);
    };
    {
      double best = -1.0;
      int bi = 0;
      for (int i = threadIdx.x; i < mr; i += kEkWG) {
        const double v = fabs(Pn[i]);
        if (v > best) { best = v; bi = i; }
      }
      wave_best(best, bi, 64);
      if (lane == 0) {
        red_v[wave] = best;
        red_i[wave] = bi;
      }
    }
    __syncthreads();
    for (int jj = 0; jj < nb; ++jj) {
      if (wave == 0) {
        double best = lane < kW ? red_v[lane] : -1.0;
        int bi = lane < kW ? red_i[lane] : mr;
        wave_best(best, bi, kW);
        const int p = __shfl(bi, 0);
        if (lane < nb) prow[lane] = Pn[p + lane * mr];
        if (lane == 0) {
          s_p = p;
          s_pv[jj] = j0 + p;
          pv[j0 + jj] = j0 + p;
          if (best == 0.0) flag[b] = 1;
        }
      }
      __syncthreads();
      const int p = s_p;
      const double d = prow[jj];
      const double inv = d != 0.0 ? 1.0 / d : 0.0;
      double nbest = -1.0;
      int nbi = jj + 1;
      for (int i = jj + 1 + threadIdx.x; i < mr; i += kEkWG) {
        double nv = 0.0;                         // this row's entry of column jj + 1 after the step
        if (i == p) {
          // row p takes the old row jj, updated; row jj takes the pivot row
          const double l = Pn[jj + jj * mr] * inv;
          for (int c = 0; c < jj; ++c) Pn[p + c * mr] = Pn[jj + c * mr];
          Pn[p + jj * mr] = l;
          for (int c = jj + 1; c < nb; ++c) {
            const double x = Pn[jj + c * mr] - l * prow[c];
            Pn[p + c * mr] = x;
            if (c == jj + 1) nv = x;
          }
          for (int c = 0; c < nb; ++c) Pn[jj + c * mr] = prow[c];
        } else {
          const double l = Pn[i + jj * mr] * inv;
          Pn[i + jj * mr] = l;
          for (int c = jj + 1; c < nb; ++c) {
            const double x = Pn[i + c * mr] - l * prow[c];
            Pn[i + c * mr] = x;
            if (c == jj + 1) nv = x;
          }
        }
        if (jj + 1 < nb) {
          const double v = fabs(nv);
          if (v > nbest) { nbest = v; nbi = i; }
        }
      }
      wave_best(nbest, nbi, 64);
      if (lane == 0) {
        red_v[wave] = nbest;
        red_i[wave] = nbi;
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < mr * nb; e += kEkWG) {
      const int i = e % mr, c = e / mr;
      A[(j0 + i) + int64_t(j0 + c) * ldo] = Pn[i + c * mr];
    }
    // the panel's interchanges as one permutation of the rows they touch,
    // composed by wave 0 (a lane per row): position sw_row[k] receives the row
    // that was at sw_src[k] (sw_row[k] < 0: unused); lanes 0 .. nb - 1 are the
    // panel's own rows, lane nb + r the pivot row of step r when it lies below
    // the panel and no earlier step chose it
    if (wave == 0) {
      auto slot_of = [&](int r) {                // the lane holding the pivot row of step r
        const int q = s_pv[r];
        if (q < j1) return q - j0;
        int f = r;
        for (int t = r - 1; t >= 0; --t)
          if (s_pv[t] == q) f = t;
        return nb + f;
      };
      int row = -1;
      if (lane < nb) {
        row = j0 + lane;
      } else if (lane < nb + nb) {
        const int r = lane - nb;
        if (s_pv[r] >= j1 && slot_of(r) == lane) row = s_pv[r];
      }
      int src = row;
      for (int r = 0; r < nb; ++r) {
        const int la = r, lb = slot_of(r);
        const int sa = __shfl(src, la), sb = __shfl(src, lb);
        if (la != lb) {
          if (lane == la) src = sb;
          else if (lane == lb) src = sa;
        }
      }
      if (lane < 2 * kP) {
        sw_row[lane] = row;
        sw_src[lane] = src;
      }
    }
    __syncthreads();
    const int ns = 2 * kP;
    const int m2 = m - j1, ldu = m2 + 1;
    // the other columns, a thread per column: gather the touched rows, scatter
    // them to their new places; right of the panel also the block row of U,
    // U12 = L11^-1 (P A)12, formed in registers and kept in LDS
    for (int c = threadIdx.x; c < m - nb; c += kEkWG) {
      const int col = c < j0 ? c : c + nb;
      double* ac = A + int64_t(col) * ldo;
      double v[2 * kP];
#pragma unroll
      for (int k = 0; k < 2 * kP; ++k)
        if (k < ns && sw_row[k] >= 0) v[k] = ac[sw_src[k]];
#pragma unroll
      for (int k = 0; k < 2 * kP; ++k)
        if (k < ns && k >= nb && sw_row[k] >= 0) ac[sw_row[k]] = v[k];
      if (col >= j1) {
#pragma unroll
        for (int r = 1; r < kP; ++r) {
          if (r >= nb) break;
          double sacc = v[r];
#pragma unroll
          for (int t = 0; t < r; ++t) sacc -= Pn[r + t * mr] * v[t];
          v[r] = sacc;
        }
      }
#pragma unroll
      for (int r = 0; r < kP; ++r)
        if (r < nb) {
          ac[j0 + r] = v[r];
          if (col >= j1) Us[(col - j1) + r * ldu] = v[r];
        }
    }
    __syncthreads();
    // trailing update A22 -= L21 U12 (rows, columns j1 .. m - 1) on the FP64
    // matrix cores, as its transpose U12^T L21^T in 16 x 16 tiles dealt
    // round-robin to the waves: lane (li, lk) holds rows i0 + li of columns
    // c0 + 4 v + lk of the tile, so each of its four loads and stores covers
    // 16 contiguous rows of four columns
    if (m2 > 0) {
      const int li = lane & 15, lk = lane >> 4;
      const int nt = (m2 + 15) / 16;
      // two tiles a wave at a time: their eight loads are issued together
      for (int t0 = wave; t0 < nt * nt; t0 += 2 * kW) {
        double old[2][4];
        int i0[2], c0[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int tile = t0 + h * kW;
          i0[h] = tile < nt * nt ? (tile % nt) * 16 : m2;      // a missing tile is all out of range
          c0[h] = tile < nt * nt ? (tile / nt) * 16 : m2;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = i0[h] + li, col = c0[h] + 4 * v + lk;
            old[h][v] = (row < m2 && col < m2) ? A[(j1 + row) + int64_t(j1 + col) * ldo] : 0.0;
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = i0[h] + li;
          hfde::hfde_d4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s4 = 0; s4 < kP / 4; ++s4) {
            const int k = 4 * s4 + lk;
            const double a = (k < nb && c0[h] + li < m2) ? Us[(c0[h] + li) + k * ldu] : 0.0;
            const double bv = (k < nb && row < m2) ? Pn[(nb + row) + k * mr] : 0.0;
            acc = hfde::mfma64(a, bv, acc);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int col = c0[h] + 4 * v + lk;
            if (row < m2 && col < m2) A[(j1 + row) + int64_t(j1 + col) * ldo] = old[h][v] - acc[v];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Columns c0 .. c0 + kEkInvCols - 1 (c0 = kEkInvCols blockIdx.x) of the
// inverse of matrix b = blockIdx.y (order m = mA for b < J, else mB) from its
// LU factors (k_ek_lu): X = P e_c, then L^-1, then U^-1, in LDS; written to
// inv + b stride (ld ldi).  Rows are taken in blocks of 16: the diagonal
// block is staged in LDS and solved by one thread per column; the rows below
// (above) it are updated by a thread per row, which loads its 16 entries of
// the factor once and applies them to every column.  15 columns a work-group
// keep X and the staged block within half a CU's LDS.
constexpr int kEkInvCols = 15;
__global__ void __launch_bounds__(256) k_ek_lu_inv(int J, int mA, int mB, const double* LU, int64_t ldo,
                                                   int64_t stride, const int32_t* piv, double* inv, int64_t ldi) {
  constexpr int kC = kEkInvCols;
  __shared__ double X[kEkMax * kC];
  __shared__ double Dg[16 * 16];               // the current diagonal block, ld 16
  const int b = blockIdx.y, c0 = blockIdx.x * kC;
  const int m = b < J ? mA : mB;
  const int nc = min(kC, m - c0);
  if (nc <= 0) return;
  const double* A = LU + int64_t(b) * stride;
  const int32_t* pv = piv + int64_t(b) * kEkMax;
  // X = P e_c: the interchanges move the unit entry of column c; its final
  // row is tracked through them
  __shared__ int s_pos[kC];
  if (threadIdx.x < nc) {
    int pos = c0 + threadIdx.x;
    for (int k = 0; k < m; ++k) {
      const int p = pv[k];
      if (pos == k) pos = p;
      else if (pos == p) pos = k;
    }
    s_pos[threadIdx.x] = pos;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * nc; e += 256) X[e] = (e % m == s_pos[e / m]) ? 1.0 : 0.0;
  // L y = x (unit lower), blocks of 16 rows top to bottom
  for (int r0 = 0; r0 < m; r0 += 16) {
    const int r1 = min(m, r0 + 16);
    {
      const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
      if (r0 + i < r1 && r0 + j < r1) Dg[i + 16 * j] = A[(r0 + i) + int64_t(r0 + j) * ldo];
    }
    __syncthreads();
    if (threadIdx.x < nc) {                    // the block's rows of this column in registers
      double* x = X + threadIdx.x * m;
      const int nr = r1 - r0;
      double xr[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) xr[r] = r < nr ? x[r0 + r] : 0.0;
#pragma unroll
      for (int r = 1; r < 16; ++r) {
        if (r >= nr) break;
        double s = xr[r];
#pragma unroll
        for (int t = 0; t < r; ++t) s -= Dg[r + 16 * t] * xr[t];
        xr[r] = s;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (r < nr) x[r0 + r] = xr[r];
    }
    __syncthreads();
    for (int i = r1 + threadIdx.x; i < m; i += 256) {
      double a[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) a[t] = r0 + t < r1 ? A[i + int64_t(r0 + t) * ldo] : 0.0;
      for (int c = 0; c < nc; ++c) {
        double* x = X + c * m;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (r0 + t < r1) s += a[t] * x[r0 + t];
        x[i] -= s;
      }
    }
    __syncthreads();
  }
  // U z = y, blocks of 16 rows bottom to top
  for (int r1 = m; r1 > 0; r1 -= 16) {
    const int r0 = max(0, r1 - 16);
    {
      const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
      if (r0 + i < r1 && r0 + j < r1) Dg[i + 16 * j] = A[(r0 + i) + int64_t(r0 + j) * ldo];
    }
    __syncthreads();
    if (threadIdx.x < nc) {                    // the block's rows of this column in registers
      double* x = X + threadIdx.x * m;
      const int nr = r1 - r0;
      double xr[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) xr[r] = r < nr ? x[r0 + r] : 0.0;
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        if (r >= nr) continue;
        double s = xr[r];
#pragma unroll
        for (int t = r + 1; t < 16; ++t)
          if (t < nr) s -= Dg[r + 16 * t] * xr[t];
        const double d = Dg[r + 16 * r];
        xr[r] = d != 0.0 ? s / d : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (r < nr) x[r0 + r] = xr[r];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r0; i += 256) {
      double a[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) a[t] = r0 + t < r1 ? A[i + int64_t(r0 + t) * ldo] : 0.0;
      for (int c = 0; c < nc; ++c) {
        double* x = X + c * m;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (r0 + t < r1) s += a[t] * x[r0 + t];
        x[i] -= s;
      }
    }
    __syncthreads();
  }
  double* out = inv + int64_t(b) * stride;
  for (int e = threadIdx.x; e < m * nc; e += 256) out[(e % m) + int64_t(c0 + e / m) * ldi] = X[e];
}

// One shift pair of the projected fADI: Z = (T_A + q I)^-1 G_in and
// Y = (T_B + p I)^-1 H_in from the explicit inverses IA, IB; K_Z gets w Z and
// K_Y gets Y (column block `off` of r <= 32 columns), G_out = G_in - w Z,
// H_out = H_in - w Y (w = p + q).  Work-groups 0 .. tA - 1 take 16-row tiles
// of the A side, the rest of the B side; in a work-group the 16 rows are
// lanes and the inner dimension is split over 16 lane groups, whose partial
// sums meet in LDS.  The inputs are read whole by every tile and the outputs
// are other buffers, so the tiles are independent.
__global__ void __launch_bounds__(256) k_ek_adi_pair(int mA, int mB, int r, double w, const double* IA,
                                                     const double* IB, int64_t ldi, const double* Gin,
                                                     const double* Hin, double* Gout, double* Hout, double* KZ,
                                                     double* KY, int64_t ldk, int off) {
  __shared__ double part[16 * 16 * 33];
  __shared__ double rin[64 * 33];             // a 64-row slice of the right-hand side
  const int tA = (mA + 15) / 16;
  const bool sa = int(blockIdx.x) < tA;
  const int tile = sa ? blockIdx.x : blockIdx.x - tA;
  const int m = sa ? mA : mB;
  const double* I = sa ? IA : IB;
  const double* in = sa ? Gin : Hin;
  double* outp = sa ? Gout : Hout;
  double* K = sa ? KZ : KY;
  const double sc = sa ? w : 1.0;
  const int rl = threadIdx.x % 16, kg = threadIdx.x / 16;
  const int i = tile * 16 + rl;
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int k0 = 0; k0 < m; k0 += 64) {
    const int kn = min(64, m - k0);
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int k = e % 64, c = e / 64;
      rin[k * 33 + c] = (k < kn && c < r) ? in[(k0 + k) + int64_t(c) * kEkMax] : 0.0;
    }
    __syncthreads();
    if (i < m) {
      for (int k = kg; k < kn; k += 16) {
        const double a = I[i + int64_t(k0 + k) * ldi];
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] += a * rin[k * 33 + c];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 32; ++c) part[(kg * 16 + rl) * 33 + c] = acc[c];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * 32; e += 256) {
    const int rr = e % 16, c = e / 16;
    const int row = tile * 16 + rr;
    if (row >= m || c >= r) continue;
    double v = 0.0;
    for (int g = 0; g < 16; ++g) v += part[(g * 16 + rr) * 33 + c];
    K[row + int64_t(off + c) * ldk] = sc * v;
    outp[row + int64_t(c) * kEkMax] = in[row + int64_t(c) * kEkMax] - w * v;
  }
}

// Per-work-group sums of squares of an m x n column-major block into part
// (gridDim.x entries), for ||X||_F.
__global__ void __launch_bounds__(256) k_ek_sumsq(int64_t m, int n, const double* X, int64_t ld, double* part) {
  __shared__ double red[256];
  const int64_t tot = m * n;
  double s = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < tot; e += int64_t(gridDim.x) * 256) {
    const double v = X[(e % m) + (e / m) * ld];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Y = E^-1 X on `cols` columns of `rows` rows (X ld ldx, Y ld ldy, distinct
// arrays): E = mass (I + mc (S + S^T)), the finite-element mass matrix, by
// its tridiagonal LU recurrence with the pivots piv (m_0 = 1, m_i = 1 -
// mc^2 / m_{i-1}, formed once on the host).  The recurrences' multipliers
// mc / m_i are at most 0.268 (mc = 1/4), so a chunk of rows can start its
// recurrence kMsWarm rows early from a zero state: the start's influence is
// below 0.268^48 ~ 4e-28 of the column's largest entry, under rounding.
// Work-group (x, y): rows [2048 x, 2048 x + 2048) of column y, its right-hand
// side, pivots and forward values staged in LDS with their halos; a thread
// per 16-row chunk, forward then backward.
constexpr int kMsTile = 2048, kMsChunk = 16, kMsWarm = 48;
__global__ void __launch_bounds__(256) k_ek_mass_solve(int64_t rows, double mass, double mc, const double* piv,
                                                       const double* X, int64_t ldx, double* Y, int64_t ldy) {
  __shared__ double bs[kMsTile + 2 * kMsWarm];   // b / mass on rows [lo, hi)
  __shared__ double ps[kMsTile + 2 * kMsWarm];   // pivots on rows [lo, hi)
  __shared__ double ys[kMsTile + kMsWarm];       // forward values on rows [t0, hi)
  const int64_t n = rows;
  const int64_t t0 = int64_t(blockIdx.x) * kMsTile, t1 = min(n, t0 + kMsTile);
  const int64_t lo = max<int64_t>(0, t0 - kMsWarm), hi = min(n, t1 + kMsWarm);
  const double* x = X + int64_t(blockIdx.y) * ldx;
  double* y = Y + int64_t(blockIdx.y) * ldy;
  const double s = 1.0 / mass;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    bs[i - lo] = s * x[i];
    ps[i - lo] = piv[i];
  }
  __syncthreads();
  const int64_t nf = (hi - t0 + kMsChunk - 1) / kMsChunk;
  for (int64_t k = threadIdx.x; k < nf; k += blockDim.x) {
    const int64_t r0 = t0 + k * kMsChunk, r1 = min(hi, r0 + kMsChunk), a = max<int64_t>(0, r0 - kMsWarm);
    double v = 0.0;
    for (int64_t i = a; i < r1; ++i) {
      v = i == a ? bs[i - lo] : bs[i - lo] - (mc / ps[i - 1 - lo]) * v;
      if (i >= r0) ys[i - t0] = v;
    }
  }
  __syncthreads();
  const int64_t nb = (t1 - t0 + kMsChunk - 1) / kMsChunk;
  for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) {
    const int64_t r0 = t0 + k * kMsChunk, r1 = min(t1, r0 + kMsChunk), e = min(n - 1, r1 - 1 + kMsWarm);
    double v = 0.0;
    for (int64_t i = e; i >= r0; --i) {
      v = i == e ? ys[i - t0] / ps[i - lo] : (ys[i - t0] - mc * v) / ps[i - lo];
      if (i < r1) y[i] = v;
    }
  }
}
