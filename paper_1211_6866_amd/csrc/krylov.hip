// Right-preconditioned Krylov solves of A~ X = R for the k columns of a block
// (Section 3 (regprob), (auxi); solver settings of Section 5).  Each column is
// an independent system; all k advance in lockstep so that every sparse
// product streams the matrix once for all columns.
//
// The caller's blocks are n x k row-major (the k values of a row are
// contiguous); BiCGStab works on n x kp copies (kp = k rounded up to even) in
// which a lane owns a pair of columns of one row.  Dot products are fused into
// the kernels that produce their operands; a one-block finisher adds the
// per-block partial sums in a fixed order (so results are deterministic) and
// updates the scalar state of every column (alpha, omega, rho, beta,
// convergence flags).
//
// BiCGStab follows van der Vorst's algorithm with r_hat = r_0.  Convergence
// is declared on the true residual rhs - A~ x, computed whenever the recursive
// residual (s at the half step, r at the full step) falls below the column's
// threshold; a failed full-step check replaces r by the true residual.  A
// breakdown (|rho|, |r_hat^T v|, |omega| or t^T t below 1e-300) restarts the
// column once with r_hat = r; a second one stops it.  ||s|| is summed with t^T s
// and t^T t (one reduction instead of two), so the half-step check runs after
// t = A M s is formed; a column that converges there takes x += alpha p_hat
// and its t is unused.  One iteration is 16 launches: 5 streaming kernels, 4
// sparse products, 2 true-residual checks that return at once unless a column
// is flagged, and 5 one-block finishers.
//
// GMRES(m) (used for the smallest workload) runs one workgroup per column for
// the whole solve: modified Gram-Schmidt Arnoldi, Givens rotations, solution
// update at the end of each cycle, convergence on the true residual.
#include "sai_internal.hpp"

#include "bicgstab_kernels.hpp"

namespace sai {
namespace {

template <int LP, class TM>
int bicgstab_lp(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R,
                double* X, const double* thr, int maxit, const Allocator& al, hipStream_t st,
                int* iters, int* status) {
  const int kp = k + (k & 1);
  const size_t nk = (size_t)n * kp;
  DBuf<double> b(&al, nk), x(&al, nk), r(&al, nk), rh(&al, nk), p(&al, nk), v(&al, nk), s(&al, nk),
      ph(&al, nk), sh(&al, nk), t(&al, nk);
  DBuf<double> sc(&al, 6 * 64);
  DBuf<int> si(&al, 10 * 64 + 8);
  DBuf<double> part(&al, (size_t)3 * NBMAX * PSTRIDE);
  HIPC(hipMemsetAsync(si.p, 0, sizeof(int) * (10 * 64 + 8), st));
  HIPC(hipMemcpyAsync(sc.p + 5 * 64, thr, sizeof(double) * k, hipMemcpyHostToDevice, st));
  State S;
  S.rho = sc.p;
  S.rho_old = sc.p + 64;
  S.alpha = sc.p + 128;
  S.omega = sc.p + 192;
  S.beta = sc.p + 256;
  S.thr = sc.p + 320;
  S.status = si.p;
  S.iters = si.p + 64;
  S.skip = si.p + 128;
  S.restarts = si.p + 192;
  S.half = si.p + 256;
  S.full = si.p + 320;
  S.rst = si.p + 384;
  S.halfconv = si.p + 448;
  S.wasact = si.p + 512;
  S.pend = si.p + 576;
  S.any = si.p + 640;
  S.part = part.p;
  Vec V{b.p, x.p, r.p, rh.p, p.p, v.p, s.p, ph.p, sh.p, t.p};
  constexpr int RPB = (64 / LP) * (NT / 64);
  // streaming kernels: a grid-stride loop over rows (fewer blocks also means
  // fewer partial sums for the finishers to add)
  const int grid = (int)std::min<int64_t>(tune_get("SGRID", 1024), (n + RPB - 1) / RPB);
  // Sparse products work on tiles of RPB rows (one per lane).  Their grid is
  // persistent: no more workgroups than fit on the device at once, so that the
  // grid sweeps the rows in one pass; it is a multiple of the XCD count.  When
  // an n x kp block fits in the 256 MB last-level (MALL) cache, XCD-contiguous
  // tile ranges let each XCD sweep one contiguous eighth of the rows and keep
  // its band of gathered rows in its own L2; larger blocks are swept by all
  // XCDs together (interleaved tiles), so that one band, not eight, must stay
  // resident in the MALL.
  const bool persist = tune_get("PERSIST", 1) != 0;
  const int xmap = tune_get("XMAP", nk * sizeof(double) <= (size_t(256) << 20) ? 1 : 0);
  auto sp_grid = [&](const void* kern) {
    const int64_t ntiles = (n + RPB - 1) / RPB;
    int64_t g = std::min<int64_t>(NBMAX, ntiles);
    if (persist) g = std::min<int64_t>(g, resident_blocks(kern, NT));
    return (int)(g >= 8 ? (g & ~int64_t(7)) : g);
  };
  // M product: gather batch sizes (CH while >= CH entries remain, then CH2)
  const int mvar = tune_get("SPMM_M", 1);
  auto spmm_m = [&](const double* Xin, double* Y) {
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(sp_grid((const void*)kern)), dim3(NT), 0, st, n, k, kp, M, Xin, Y,
                         S, xmap);
    };
    switch (mvar) {
      case 0: go(k_spmm<LP, TM, 8, 4>); break;
      case 2: go(k_spmm<LP, TM, 5, 0>); break;
      case 3: go(k_spmm<LP, TM, 16, 8>); break;
      default: go(k_spmm<LP, TM, 6, 3>); break;
    }
  };
  // A~ products (with their dot products): gather batch sizes
  const int avar = tune_get("SPMM_A", 0);
  const void* kav = avar == 1 ? (const void*)k_av<LP, 8, 4>
                    : avar == 2 ? (const void*)k_av<LP, 7, 0> : (const void*)k_av<LP, 4, 2>;
  const void* kat = avar == 1 ? (const void*)k_at<LP, 8, 4>
                    : avar == 2 ? (const void*)k_at<LP, 7, 0> : (const void*)k_at<LP, 4, 2>;
  const int tgrid = std::min(sp_grid(kav), sp_grid(kat));
  auto spmm_av = [&]() {
    if (avar == 1) hipLaunchKernelGGL((k_av<LP, 8, 4>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
    else if (avar == 2) hipLaunchKernelGGL((k_av<LP, 7, 0>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
    else hipLaunchKernelGGL((k_av<LP, 4, 2>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
  };
  auto spmm_at = [&]() {
    if (avar == 1) hipLaunchKernelGGL((k_at<LP, 8, 4>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
    else if (avar == 2) hipLaunchKernelGGL((k_at<LP, 7, 0>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
    else hipLaunchKernelGGL((k_at<LP, 4, 2>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
  };
  {
    SAI_PROF("bicg_init", st);
    hipLaunchKernelGGL((k_init<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, R, V, S);
    hipLaunchKernelGGL((k_fin<1, F_INIT>), dim3(1), dim3(FNT), 0, st, k, S, grid, 0, 0);
  }
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, st, k, S, 0, maxit);
  LAUNCH_CHECK();
  // The active-column count of iteration it is read back while iteration it+1
  // runs (two pinned slots, one event each), so the device never waits for the
  // host.  An iteration queued after the last column stopped finds no active
  // column and does no work.
  HostStage hs(16);
  int* slot = hs.as<int>();
  hipEvent_t ev[2];
  HIPC(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIPC(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } evg{ev};
  HIPC(hipMemcpyAsync(slot, S.any + 3, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipEventRecord(ev[0], st));
  HIPC(hipEventSynchronize(ev[0]));
  bool go_on = slot[0] > 0;
  for (int it = 1; it <= maxit && go_on; ++it) {
#define LK(name, ...)              \
  do {                             \
    SAI_PROF(name, st);            \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)
    constexpr bool MF = sizeof(TM) == 4;
    LK("bicg_p_update", (k_pupdate<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    {
      SAI_PROF(MF ? "bicg_spmm_M_f32" : "bicg_spmm_M_f64", st);
      spmm_m(V.p, V.ph);
    }
    {
      SAI_PROF("bicg_spmm_A_dot1", st);
      spmm_av();
    }
    LK("bicg_finish", (k_fin<1, F_AV>), dim3(1), dim3(FNT), 0, st, k, S, tgrid, 0, 0);
    LK("bicg_s_update", (k_s<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    {
      SAI_PROF(MF ? "bicg_spmm_M_f32" : "bicg_spmm_M_f64", st);
      spmm_m(V.s, V.sh);
    }
    {
      SAI_PROF("bicg_spmm_A_dot2", st);
      spmm_at();
    }
    LK("bicg_finish", (k_fin<3, F_AT>), dim3(1), dim3(FNT), 0, st, k, S, tgrid, 0, 0);
    LK("bicg_halfcheck", (k_halfcheck<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, A, V, S);
    LK("bicg_finish", (k_fin<1, F_HALF>), dim3(1), dim3(FNT), 0, st, k, S, grid, 0, 0);
    LK("bicg_xr_update", (k_xr<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    LK("bicg_finish", (k_fin<2, F_XR>), dim3(1), dim3(FNT), 0, st, k, S, grid, 0, 0);
    LK("bicg_fullcheck", (k_fullcheck<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, A, V, S);
    LK("bicg_finish", (k_fin<2, F_FULL>), dim3(1), dim3(FNT), 0, st, k, S, grid, 0, 0);
    LK("bicg_restart", (k_restart<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    LK("bicg_finish_end", (k_fin<1, F_RESTART_END>), dim3(1), dim3(FNT), 0, st, k, S, grid, it, maxit);
#undef LK
    LAUNCH_CHECK();
    HIPC(hipMemcpyAsync(slot + (it & 1), S.any + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipEventRecord(ev[it & 1], st));
    if (it > 1) {
      // count after iteration it-1 (iteration it is already queued behind it)
      HIPC(hipEventSynchronize(ev[(it - 1) & 1]));
      go_on = slot[(it - 1) & 1] > 0;
    }
  }
  hipLaunchKernelGGL((k_copy_out<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V.x, X);
  LAUNCH_CHECK();
  std::vector<int> hst(k), hit(k);
  HIPC(hipMemcpyAsync(hst.data(), S.status, sizeof(int) * k, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(hit.data(), S.iters, sizeof(int) * k, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  int worst = SAI_OK;
  for (int c = 0; c < k; ++c) {
    int code = hst[c] == ST_CONV ? 0 : (hst[c] == ST_BREAK ? 2 : 1);
    if (status) status[c] = code;
    if (iters) iters[c] = hit[c];
    if (code == 2) worst = SAI_EBREAKDOWN;
    else if (code == 1 && worst == SAI_OK) worst = SAI_ENOCONV;
  }
  return worst;
}

// ---- GMRES(m): one workgroup per column -------------------------------------------

constexpr int GM_NT = 1024;
constexpr int GM_MAXM = 64;

__device__ double gm_block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < GM_NT / WAVE; ++i) s += red[i];
  __syncthreads();
  return s;
}

template <class TM>
__global__ void __launch_bounds__(GM_NT) k_gmres(int64_t n, int k, Csr<double> A, Csr<TM> M,
                                                 const double* R, double* X, const double* thr_d,
                                                 int m, int maxit, double* work, int* iters,
                                                 int* status) {
  __shared__ double H[(GM_MAXM + 1) * GM_MAXM];
  __shared__ double g[GM_MAXM + 1], cs[GM_MAXM], sn[GM_MAXM], y[GM_MAXM];
  __shared__ double red[GM_NT / WAVE];
  __shared__ int flag;
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const double thr = thr_d[c];
  double* Vb = work + (int64_t)c * (m + 3) * n;  // m+1 basis vectors, then z, w
  double* z = Vb + (int64_t)(m + 1) * n;
  double* w = z + n;
  // x = 0, r = rhs
  double acc = 0.0;
  for (int64_t i = tid; i < n; i += GM_NT) {
    X[i * k + c] = 0.0;
    const double b = R[i * k + c];
    w[i] = b;
    acc += b * b;
  }
  double beta = sqrt(gm_block_sum(acc, red));
  int it = 0, st = ST_ACTIVE;
  if (beta < thr) st = ST_CONV;
  while (st == ST_ACTIVE && it < maxit) {
    for (int64_t i = tid; i < n; i += GM_NT) Vb[i] = w[i] / beta;
    if (tid == 0) {
      g[0] = beta;
      for (int q = 1; q <= m; ++q) g[q] = 0.0;
    }
    __syncthreads();
    int kk = 0;
    for (int j = 0; j < m; ++j) {
      ++it;
      const double* vj = Vb + (int64_t)j * n;
      for (int64_t i = tid; i < n; i += GM_NT) {
        double s = 0.0;
        for (int32_t e = M.rp[i]; e < M.rp[i + 1]; ++e) s += (double)M.v[e] * vj[M.ci[e]];
        z[i] = s;
      }
      __syncthreads();
      for (int64_t i = tid; i < n; i += GM_NT) {
        double s = 0.0;
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) s += A.v[e] * z[A.ci[e]];
        w[i] = s;
      }
      __syncthreads();
      for (int q = 0; q <= j; ++q) {  // modified Gram-Schmidt
        const double* vq = Vb + (int64_t)q * n;
        double d = 0.0;
        for (int64_t i = tid; i < n; i += GM_NT) d += w[i] * vq[i];
        d = gm_block_sum(d, red);
        for (int64_t i = tid; i < n; i += GM_NT) w[i] -= d * vq[i];
        if (tid == 0) H[q * GM_MAXM + j] = d;
        __syncthreads();
      }
      double nn = 0.0;
      for (int64_t i = tid; i < n; i += GM_NT) nn += w[i] * w[i];
      const double hnext = sqrt(gm_block_sum(nn, red));
      if (tid == 0) {
        H[(j + 1) * GM_MAXM + j] = hnext;
        for (int q = 0; q < j; ++q) {
          const double a = H[q * GM_MAXM + j], b = H[(q + 1) * GM_MAXM + j];
          H[q * GM_MAXM + j] = cs[q] * a + sn[q] * b;
          H[(q + 1) * GM_MAXM + j] = -sn[q] * a + cs[q] * b;
        }
        const double a = H[j * GM_MAXM + j], b = H[(j + 1) * GM_MAXM + j];
        double cc = 1.0, ss = 0.0;
        if (b != 0.0) {
          const double h = hypot(a, b);
          cc = a / h;
          ss = b / h;
        }
        cs[j] = cc;
        sn[j] = ss;
        H[j * GM_MAXM + j] = cc * a + ss * b;
        H[(j + 1) * GM_MAXM + j] = 0.0;
        g[j + 1] = -ss * g[j];
        g[j] = cc * g[j];
        flag = (hnext == 0.0 || fabs(g[j + 1]) < thr || it >= maxit) ? 1 : 0;
      }
      __syncthreads();
      kk = j + 1;
      if (flag) break;
      double* vn = Vb + (int64_t)(j + 1) * n;
      for (int64_t i = tid; i < n; i += GM_NT) vn[i] = w[i] / hnext;
      __syncthreads();
    }
    if (tid == 0) {
      for (int q = kk - 1; q >= 0; --q) {
        double s = g[q];
        for (int u = q + 1; u < kk; ++u) s -= H[q * GM_MAXM + u] * y[u];
        y[q] = s / H[q * GM_MAXM + q];
      }
    }
    __syncthreads();
    for (int64_t i = tid; i < n; i += GM_NT) {
      double s = 0.0;
      for (int q = 0; q < kk; ++q) s += y[q] * Vb[(int64_t)q * n + i];
      w[i] = s;
    }
    __syncthreads();
    for (int64_t i = tid; i < n; i += GM_NT) {
      double s = 0.0;
      for (int32_t e = M.rp[i]; e < M.rp[i + 1]; ++e) s += (double)M.v[e] * w[M.ci[e]];
      X[i * k + c] += s;
    }
    __syncthreads();
    acc = 0.0;
    for (int64_t i = tid; i < n; i += GM_NT) {
      double s = 0.0;
      for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) s += A.v[e] * X[(int64_t)A.ci[e] * k + c];
      const double rv = R[i * k + c] - s;
      w[i] = rv;
      acc += rv * rv;
    }
    beta = sqrt(gm_block_sum(acc, red));
    if (beta < thr) st = ST_CONV;
  }
  if (st == ST_ACTIVE) st = ST_MAXIT;
  if (tid == 0) {
    iters[c] = it;
    status[c] = st;
  }
}

template <class TM>
int gmres_run(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R, double* X,
              const double* thr, int restart, int maxit, const Allocator& al, hipStream_t st,
              int* iters, int* status) {
  if (restart < 1 || restart > GM_MAXM) SAI_THROW(SAI_EINVAL, "GMRES restart must be in [1, %d]", GM_MAXM);
  DBuf<double> work(&al, (size_t)k * (restart + 3) * n);
  DBuf<double> dthr(&al, k);
  DBuf<int> dit(&al, k), dst(&al, k);
  HIPC(hipMemcpyAsync(dthr.p, thr, sizeof(double) * k, hipMemcpyHostToDevice, st));
  SAI_PROF("gmres_fused", st);
  hipLaunchKernelGGL((k_gmres<TM>), dim3(k), dim3(GM_NT), 0, st, n, k, A, M, R, X, dthr.p, restart,
                     maxit, work.p, dit.p, dst.p);
  LAUNCH_CHECK();
  std::vector<int> hst(k), hit(k);
  HIPC(hipMemcpyAsync(hst.data(), dst.p, sizeof(int) * k, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(hit.data(), dit.p, sizeof(int) * k, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  int worst = SAI_OK;
  for (int c = 0; c < k; ++c) {
    const int code = hst[c] == ST_CONV ? 0 : 1;
    if (status) status[c] = code;
    if (iters) iters[c] = hit[c];
    if (code) worst = SAI_ENOCONV;
  }
  return worst;
}

template <class TM>
int krylov_typed(const sai_split_s* sp, const sai_precond_s* pc, int transpose, int k,
                 const double* R, double* X, const double* thr, const sai_solve_opts& o,
                 hipStream_t st, int* iters, int* status) {
  const Allocator al{sp->al.a, st};
  Csr<double> A;
  Csr<TM> M;
  if (!transpose) {
    A = {sp->t_row_ptr.p, sp->t_col_idx.p, sp->t_val.p};
    M = {pc->row_ptr.p, pc->col_idx.p, (const TM*)pc->val.p};
  } else {
    A = {sp->t_col_ptr.p, sp->t_row_idx.p, sp->t_cval.p};
    M = {pc->col_ptr.p, pc->row_idx.p, (const TM*)pc->cval.p};
  }
  const int64_t n = sp->n;
  if (o.method == SAI_GMRES)
    return gmres_run<TM>(A, M, n, k, R, X, thr, o.restart, o.maxit, al, st, iters, status);
  // lanes per row: the smallest of 1, 2, 4, 6, 8, 12, 16, 32 covering the pairs
  const int pairs = (k + 1) / 2;
  if (pairs <= 1) return bicgstab_lp<1, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (pairs <= 2) return bicgstab_lp<2, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (pairs <= 4) return bicgstab_lp<4, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (pairs <= 6) return bicgstab_lp<6, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (pairs <= 8) return bicgstab_lp<8, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (pairs <= 12) return bicgstab_lp<12, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (pairs <= 16) return bicgstab_lp<16, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  return bicgstab_lp<32, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
}

}  // namespace

int krylov_impl(const sai_split_s* sp, const sai_precond_s* pc, int transpose, int k,
                const double* R, double* X, const double* thr, const sai_solve_opts& o,
                hipStream_t st, int32_t* iters, int32_t* status) {
  if (k < 1 || k > 64) SAI_THROW(SAI_EINVAL, "k must be in [1, 64] (got %d)", k);
  if (o.method != SAI_BICGSTAB && o.method != SAI_GMRES) SAI_THROW(SAI_EINVAL, "bad method");
  if (o.maxit < 0) SAI_THROW(SAI_EINVAL, "maxit < 0");
  if (pc->n != sp->n) SAI_THROW(SAI_EINVAL, "preconditioner and split sizes differ");
  if (pc->precision == SAI_FP32)
    return krylov_typed<float>(sp, pc, transpose, k, R, X, thr, o, st, iters, status);
  return krylov_typed<double>(sp, pc, transpose, k, R, X, thr, o, st, iters, status);
}

}  // namespace sai
