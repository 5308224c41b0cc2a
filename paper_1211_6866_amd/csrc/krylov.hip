// Right-preconditioned Krylov solves of A~ X = R for the k columns of a block
// (Section 3 (regprob), (auxi); solver settings of Section 5).  Each column is
// an independent system; all k advance in lockstep so that every sparse
// product streams the matrix once for all columns.
//
// Blocks are n x k row-major (the k values of a row are contiguous).  A group
// of GK lanes (GK = next power of two >= k) handles one row; lane c owns
// column c.  Dot products are fused into the kernels that produce their
// operands; the per-block partial sums are reduced by the last block to finish
// (fixed order, so results are deterministic), which then updates the scalar
// state of every column (alpha, omega, rho, beta, convergence flags).
//
// BiCGStab follows van der Vorst's algorithm with r_hat = r_0.  Convergence
// is declared on the true residual rhs - A~ x, computed whenever the recursive
// residual (s at the half step, r at the full step) falls below the column's
// threshold; a failed full-step check replaces r by the true residual.  A
// breakdown (|rho|, |r_hat^T v|, |omega| or t^T t below 1e-300) restarts the
// column once with r_hat = r; a second one stops it.
//
// GMRES(m) (used for the smallest workload) runs one workgroup per column for
// the whole solve: modified Gram-Schmidt Arnoldi, Givens rotations, solution
// update at the end of each cycle, convergence on the true residual.
#include "sai_internal.hpp"

namespace sai {
namespace {

constexpr int NT = 256;
constexpr int NB = 1024;
constexpr double TINY = 1e-300;

enum { ST_ACTIVE = 0, ST_CONV = 1, ST_MAXIT = 2, ST_BREAK = 3 };

template <class TV>
struct Csr {
  const int32_t* rp;
  const int32_t* ci;
  const TV* v;
};

struct State {
  double *rho, *rho_old, *alpha, *omega, *beta, *thr;
  int *status, *iters, *skip, *restarts, *half, *full, *rst, *halfconv, *wasact;
  int* any;  // 0 half, 1 full, 2 restart, 3 active count, 4 half-converged
  double* part;
  unsigned* counter;
};

struct Vec {
  const double* rhs;
  double *x, *r, *rh, *p, *v, *s, *ph, *sh, *t;
};

__device__ __forceinline__ bool col_active(const State& S, int c) {
  return S.status[c] == ST_ACTIVE && S.skip[c] == 0;
}

template <class TV>
__device__ __forceinline__ double row_prod(const Csr<TV>& A, int64_t i, const double* X, int k,
                                           int c) {
  double acc = 0.0;
  const int32_t e1 = A.rp[i + 1];
  int32_t e = A.rp[i];
  for (; e + 1 < e1; e += 2) {
    const int32_t j0 = A.ci[e], j1 = A.ci[e + 1];
    const double v0 = (double)A.v[e], v1 = (double)A.v[e + 1];
    const double x0 = X[(int64_t)j0 * k + c], x1 = X[(int64_t)j1 * k + c];
    acc += v0 * x0;
    acc += v1 * x1;
  }
  if (e < e1) acc += (double)A.v[e] * X[(int64_t)A.ci[e] * k + c];
  return acc;
}

// Block-reduce ND per-lane accumulators (per column), publish the block's
// partials, and let the last block to finish form the totals in tot[d][c].
// Returns true in the last block (all threads).
template <int GK, int ND>
__device__ bool reduce_dots(double (&acc)[ND], const State& S, double (*tot)[GK]) {
  constexpr int RPB = NT / GK;
  __shared__ double red[ND][NT];
  __shared__ bool last;
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < ND; ++d) red[d][t] = acc[d];
  __syncthreads();
  if (t < GK) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s = 0.0;
      for (int r = 0; r < RPB; ++r) s += red[d][r * GK + t];
      S.part[((int64_t)d * NB + blockIdx.x) * GK + t] = s;
    }
  }
  __threadfence();
  __syncthreads();
  if (t == 0) last = (atomicAdd(S.counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const int c = t % GK, q = t / GK;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s = 0.0;
    for (int b = q; b < (int)gridDim.x; b += RPB)
      s += __builtin_nontemporal_load(&S.part[((int64_t)d * NB + b) * GK + c]);
    red[d][t] = s;
  }
  __syncthreads();
  if (t < GK) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s = 0.0;
      for (int r = 0; r < RPB; ++r) s += red[d][r * GK + t];
      tot[d][t] = s;
    }
  }
  if (t == 0) *S.counter = 0u;
  __syncthreads();
  return true;
}

#define ROW_LOOP                                                  \
  constexpr int RPB = NT / GK;                                    \
  const int c = threadIdx.x % GK;                                 \
  const bool lane_ok = c < k;                                     \
  for (int64_t i = (int64_t)blockIdx.x * RPB + threadIdx.x / GK; i < n; \
       i += (int64_t)gridDim.x * RPB)

// ---- initialisation: x = 0, r = r_hat = rhs, p = v = 0, rho = ||r||^2 ----------
template <int GK>
__global__ void __launch_bounds__(NT) k_init(int64_t n, int k, Vec V, State S) {
  double acc[1] = {0.0};
  ROW_LOOP {
    if (!lane_ok) continue;
    const int64_t q = i * k + c;
    const double b = V.rhs[q];
    V.x[q] = 0.0;
    V.r[q] = b;
    V.rh[q] = b;
    V.p[q] = 0.0;
    V.v[q] = 0.0;
    acc[0] += b * b;
  }
  __shared__ double tot[1][GK];
  if (!reduce_dots<GK, 1>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k) {
    const double rr = tot[0][t];
    S.rho[t] = rr;
    S.rho_old[t] = 1.0;
    S.alpha[t] = 1.0;
    S.omega[t] = 1.0;
    S.beta[t] = rr;
    S.skip[t] = 0;
    S.restarts[t] = 0;
    S.half[t] = S.full[t] = S.rst[t] = S.halfconv[t] = 0;
    S.iters[t] = 0;
    S.status[t] = (sqrt(rr) < S.thr[t]) ? ST_CONV : ST_ACTIVE;
  }
  if (t == 0) { S.any[0] = S.any[1] = S.any[2] = S.any[4] = 0; }
}

// ---- p = r + beta (p - omega v) -------------------------------------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_pupdate(int64_t n, int k, Vec V, State S) {
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c)) continue;
    const int64_t q = i * k + c;
    V.p[q] = V.r[q] + S.beta[c] * (V.p[q] - S.omega[c] * V.v[q]);
  }
}

// ---- Y = Op X (plain product; columns not active are skipped) ---------------------
template <int GK, class TV>
__global__ void __launch_bounds__(NT) k_spmm(int64_t n, int k, Csr<TV> A, const double* X,
                                             double* Y, State S) {
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c)) continue;
    Y[i * k + c] = row_prod(A, i, X, k, c);
  }
}

// ---- v = A p_hat, sigma = r_hat^T v, alpha = rho / sigma --------------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_av(int64_t n, int k, Csr<double> A, Vec V, State S) {
  double acc[1] = {0.0};
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c)) continue;
    const double y = row_prod(A, i, V.ph, k, c);
    V.v[i * k + c] = y;
    acc[0] += V.rh[i * k + c] * y;
  }
  __shared__ double tot[1][GK];
  if (!reduce_dots<GK, 1>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && col_active(S, t)) {
    const double sig = tot[0][t];
    if (fabs(sig) < TINY) {
      S.skip[t] = 1;
      S.rst[t] = 1;
      S.any[2] = 1;
    } else {
      S.alpha[t] = S.rho[t] / sig;
    }
  }
}

// ---- s = r - alpha v, half-step flag when ||s|| < thr --------------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_s(int64_t n, int k, Vec V, State S) {
  double acc[1] = {0.0};
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c)) continue;
    const int64_t q = i * k + c;
    const double sv = V.r[q] - S.alpha[c] * V.v[q];
    V.s[q] = sv;
    acc[0] += sv * sv;
  }
  __shared__ double tot[1][GK];
  if (!reduce_dots<GK, 1>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && col_active(S, t)) {
    if (sqrt(tot[0][t]) < S.thr[t]) {
      S.half[t] = 1;
      S.any[0] = 1;
    }
  }
}

// ---- half-step true residual: rhs - A (x + alpha p_hat) for flagged columns -------
template <int GK>
__global__ void __launch_bounds__(NT) k_halfcheck(int64_t n, int k, Csr<double> A, Vec V, State S) {
  if (S.any[0] == 0) return;
  double acc[1] = {0.0};
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c) || !S.half[c]) continue;
    const double al = S.alpha[c];
    double y = 0.0;
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int64_t q = (int64_t)A.ci[e] * k + c;
      y += A.v[e] * (V.x[q] + al * V.ph[q]);
    }
    const double rt = V.rhs[i * k + c] - y;
    acc[0] += rt * rt;
  }
  __shared__ double tot[1][GK];
  if (!reduce_dots<GK, 1>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && col_active(S, t) && S.half[t]) {
    if (sqrt(tot[0][t]) < S.thr[t]) {
      S.halfconv[t] = 1;
      S.any[4] = 1;
    }
  }
}

// ---- x += alpha p_hat for the columns that converged at the half step -------------
template <int GK>
__global__ void __launch_bounds__(NT) k_halfapply(int64_t n, int k, Vec V, State S, int it) {
  if (S.any[4] == 0) return;
  ROW_LOOP {
    if (!lane_ok || !S.halfconv[c] || S.status[c] != ST_ACTIVE) continue;
    const int64_t q = i * k + c;
    V.x[q] += S.alpha[c] * V.ph[q];
  }
}

// ---- t = A s_hat, omega = t^T s / t^T t -----------------------------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_at(int64_t n, int k, Csr<double> A, Vec V, State S) {
  double acc[2] = {0.0, 0.0};
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c) || S.halfconv[c]) continue;
    const double y = row_prod(A, i, V.sh, k, c);
    V.t[i * k + c] = y;
    acc[0] += y * V.s[i * k + c];
    acc[1] += y * y;
  }
  __shared__ double tot[2][GK];
  if (!reduce_dots<GK, 2>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && col_active(S, t) && !S.halfconv[t]) {
    const double tt = tot[1][t];
    if (tt < TINY) {
      S.skip[t] = 1;
      S.rst[t] = 1;
      S.any[2] = 1;
    } else {
      S.omega[t] = tot[0][t] / tt;
    }
  }
}

// ---- x += alpha p_hat + omega s_hat, r = s - omega t, rho_new = r_hat^T r -----------
template <int GK>
__global__ void __launch_bounds__(NT) k_xr(int64_t n, int k, Vec V, State S) {
  double acc[2] = {0.0, 0.0};
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c) || S.halfconv[c]) continue;
    const int64_t q = i * k + c;
    V.x[q] += S.alpha[c] * V.ph[q] + S.omega[c] * V.sh[q];
    const double rv = V.s[q] - S.omega[c] * V.t[q];
    V.r[q] = rv;
    acc[0] += V.rh[q] * rv;
    acc[1] += rv * rv;
  }
  __shared__ double tot[2][GK];
  if (!reduce_dots<GK, 2>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && col_active(S, t) && !S.halfconv[t]) {
    const double rho_new = tot[0][t];
    S.rho_old[t] = S.rho[t];
    S.rho[t] = rho_new;
    S.beta[t] = (rho_new / S.rho_old[t]) * (S.alpha[t] / S.omega[t]);
    if (sqrt(tot[1][t]) < S.thr[t]) {
      S.full[t] = 1;
      S.any[1] = 1;  // breakdown checks follow the true-residual check
    } else if (fabs(S.omega[t]) < TINY || fabs(rho_new) < TINY) {
      S.rst[t] = 1;
      S.any[2] = 1;
    }
  }
}

// ---- full-step true residual; replaces r when it does not pass --------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_fullcheck(int64_t n, int k, Csr<double> A, Vec V, State S) {
  if (S.any[1] == 0) return;
  double acc[2] = {0.0, 0.0};
  ROW_LOOP {
    if (!lane_ok || !col_active(S, c) || !S.full[c]) continue;
    const int64_t q = i * k + c;
    const double rt = V.rhs[q] - row_prod(A, i, V.x, k, c);
    V.r[q] = rt;
    acc[0] += rt * rt;
    acc[1] += V.rh[q] * rt;
  }
  __shared__ double tot[2][GK];
  if (!reduce_dots<GK, 2>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && col_active(S, t) && S.full[t]) {
    if (sqrt(tot[0][t]) < S.thr[t]) {
      S.status[t] = ST_CONV;  // iteration count set at the end of the iteration
    } else {
      const double rho_new = tot[1][t];
      S.rho[t] = rho_new;
      S.beta[t] = (rho_new / S.rho_old[t]) * (S.alpha[t] / S.omega[t]);
      if (fabs(S.omega[t]) < TINY || fabs(rho_new) < TINY) {
        S.rst[t] = 1;
        S.any[2] = 1;
      }
    }
  }
}

// ---- restart: r_hat = r, p = v = 0, rho = r^T r ----------------------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_restart(int64_t n, int k, Vec V, State S) {
  if (S.any[2] == 0) return;
  double acc[1] = {0.0};
  ROW_LOOP {
    if (!lane_ok || !S.rst[c] || S.status[c] != ST_ACTIVE) continue;
    const int64_t q = i * k + c;
    const double rv = V.r[q];
    V.rh[q] = rv;
    V.p[q] = 0.0;
    V.v[q] = 0.0;
    acc[0] += rv * rv;
  }
  __shared__ double tot[1][GK];
  if (!reduce_dots<GK, 1>(acc, S, tot)) return;
  const int t = threadIdx.x;
  if (t < k && S.rst[t] && S.status[t] == ST_ACTIVE) {
    const double rr = tot[0][t];
    S.rho[t] = rr;
    S.rho_old[t] = S.alpha[t] = S.omega[t] = 1.0;
    S.beta[t] = rr;
    S.restarts[t] += 1;
    if (S.restarts[t] > 1) S.status[t] = ST_BREAK;
  }
}

// ---- end of an iteration: record iterations, clear flags, count active columns ----
__global__ void k_iter_end(int k, State S, int it, int maxit) {
  __shared__ int cnt;
  const int t = threadIdx.x;
  if (t == 0) cnt = 0;
  __syncthreads();
  if (t < k) {
    int st = S.status[t];
    if (S.halfconv[t] && st == ST_ACTIVE) st = ST_CONV;
    if (it > 0 && S.wasact[t]) S.iters[t] = it;
    if (st == ST_ACTIVE && it >= maxit) st = ST_MAXIT;
    S.status[t] = st;
    S.wasact[t] = (st == ST_ACTIVE) ? 1 : 0;
    S.skip[t] = 0;
    S.half[t] = S.full[t] = S.rst[t] = S.halfconv[t] = 0;
    if (st == ST_ACTIVE) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (t == 0) {
    S.any[0] = S.any[1] = S.any[2] = S.any[4] = 0;
    S.any[3] = cnt;
  }
}

template <int GK, class TM>
int bicgstab_gk(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R,
                double* X, const double* thr, int maxit, const Allocator& al, hipStream_t st,
                int* iters, int* status) {
  const size_t nk = (size_t)n * k;
  DBuf<double> r(&al, nk), rh(&al, nk), p(&al, nk), v(&al, nk), s(&al, nk), ph(&al, nk),
      sh(&al, nk), t(&al, nk);
  DBuf<double> sc(&al, 6 * 64);
  DBuf<int> si(&al, 9 * 64 + 8);
  DBuf<double> part(&al, (size_t)2 * NB * GK);
  DBuf<unsigned> counter(&al, 1);
  HIPC(hipMemsetAsync(counter.p, 0, sizeof(unsigned), st));
  HIPC(hipMemsetAsync(si.p, 0, sizeof(int) * (9 * 64 + 8), st));
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
  S.any = si.p + 576;
  S.part = part.p;
  S.counter = counter.p;
  Vec V{R, X, r.p, rh.p, p.p, v.p, s.p, ph.p, sh.p, t.p};
  constexpr int RPB = NT / GK;
  const unsigned grid = (unsigned)std::min<int64_t>(NB, (n + RPB - 1) / RPB);
  HostStage hs(16);
  hipLaunchKernelGGL((k_init<GK>), dim3(grid), dim3(NT), 0, st, n, k, V, S);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, st, k, S, 0, maxit);
  LAUNCH_CHECK();
  HIPC(hipMemcpyAsync(hs.p, S.any + 3, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  int active = *hs.as<int>();
  for (int it = 1; it <= maxit && active > 0; ++it) {
    hipLaunchKernelGGL((k_pupdate<GK>), dim3(grid), dim3(NT), 0, st, n, k, V, S);
    hipLaunchKernelGGL((k_spmm<GK, TM>), dim3(grid), dim3(NT), 0, st, n, k, M, (const double*)V.p, V.ph, S);
    hipLaunchKernelGGL((k_av<GK>), dim3(grid), dim3(NT), 0, st, n, k, A, V, S);
    hipLaunchKernelGGL((k_s<GK>), dim3(grid), dim3(NT), 0, st, n, k, V, S);
    hipLaunchKernelGGL((k_halfcheck<GK>), dim3(grid), dim3(NT), 0, st, n, k, A, V, S);
    hipLaunchKernelGGL((k_halfapply<GK>), dim3(grid), dim3(NT), 0, st, n, k, V, S, it);
    hipLaunchKernelGGL((k_spmm<GK, TM>), dim3(grid), dim3(NT), 0, st, n, k, M, (const double*)V.s, V.sh, S);
    hipLaunchKernelGGL((k_at<GK>), dim3(grid), dim3(NT), 0, st, n, k, A, V, S);
    hipLaunchKernelGGL((k_xr<GK>), dim3(grid), dim3(NT), 0, st, n, k, V, S);
    hipLaunchKernelGGL((k_fullcheck<GK>), dim3(grid), dim3(NT), 0, st, n, k, A, V, S);
    hipLaunchKernelGGL((k_restart<GK>), dim3(grid), dim3(NT), 0, st, n, k, V, S);
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, st, k, S, it, maxit);
    LAUNCH_CHECK();
    HIPC(hipMemcpyAsync(hs.p, S.any + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    active = *hs.as<int>();
  }
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
  if (k <= 4) return bicgstab_gk<4, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (k <= 8) return bicgstab_gk<8, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (k <= 16) return bicgstab_gk<16, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  if (k <= 32) return bicgstab_gk<32, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
  return bicgstab_gk<64, TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status);
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
