// Kernels of the batched right-preconditioned BiCGStab (included by krylov.hip).
//
// Blocks are n x k row-major.  A group of GK lanes (GK = next power of two >= k)
// handles one row, lane c owning column c; a 256-thread block covers RPB =
// 256/GK rows at a time.  Sparse products stage the column indices and values
// of a tile of SUB*RPB consecutive rows in LDS with one coalesced copy, then
// every lane gathers X[j, c] for up to eight entries at a time, so that eight
// independent loads are in flight.  Per-column state (status, scalars) is read
// once per kernel.  Dot products are reduced per block into partials; a
// one-block finisher kernel adds the partials in a fixed order
// (deterministic) and updates the per-column scalars and flags.
#pragma once

namespace sai {
namespace {

constexpr int NT = 256;
constexpr int NBMAX = 2048;
constexpr int SUB = 4;
constexpr int CAP_A = 1024;  // staged entries per tile: A~ (about 7 per row)
constexpr int CAP_M = 3072;  // and M (about 25 per row)
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
};

struct Vec {
  const double* rhs;
  double *x, *r, *rh, *p, *v, *s, *ph, *sh, *t;
  // FP32 copies of p and s written beside them (null: not kept); the FP32
  // preconditioner is applied to these copies
  float *pf, *sf;
};

__device__ __forceinline__ bool col_on(const State& S, int c, int k) {
  return c < k && S.status[c] == ST_ACTIVE && S.skip[c] == 0;
}

// sum_e A_ie X[j_e, c] over entries eb..ee of (sci, sv), accumulated in FP64
// (a product of two FP32 numbers is exact in FP64)
template <class TV, class XT>
__device__ __forceinline__ double row_prod_lds(const int32_t* __restrict__ sci,
                                               const TV* __restrict__ sv, int eb, int ee,
                                               const XT* __restrict__ X, int k, int c) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int e = eb;
  for (; e + 7 < ee; e += 8) {
    XT x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = X[(int64_t)sci[e + u] * k + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += (double)sv[e + u] * (double)x[u];
  }
  if (e + 3 < ee) {
    XT x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = X[(int64_t)sci[e + u] * k + c];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] += (double)sv[e + u] * (double)x[u];
    e += 4;
  }
  for (; e < ee; ++e) a[4] += (double)sv[e] * (double)X[(int64_t)sci[e] * k + c];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

template <class TV, class XT>
__device__ __forceinline__ double row_prod(const Csr<TV>& A, int64_t i, const XT* __restrict__ X,
                                           int k, int c) {
  return row_prod_lds<TV, XT>(A.ci, A.v, A.rp[i], A.rp[i + 1], X, k, c);
}

// SI rows at once, entries eb[q]..ee[q] in LDS: the gathers of the first CH
// entries of every row are all issued before any is consumed (SI*CH loads in
// flight per lane); entries past CH follow in a plain loop.  BF (branch-free):
// a slot past the row's end loads row 0 of X (a valid address) and is
// multiplied by zero, so that the compiler issues every load before the first
// wait; otherwise each slot is guarded, which suits short rows (A~).
template <class TV, int CH, int SI, bool BF, class XT>
__device__ __forceinline__ void rows_prod_batch(const int32_t* __restrict__ sci,
                                                const TV* __restrict__ sv, const int (&eb)[SI],
                                                const int (&ee)[SI], const XT* __restrict__ X,
                                                int k, int c, double (&out)[SI]) {
  XT xv[SI][CH];
#pragma unroll
  for (int q = 0; q < SI; ++q) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = eb[q] + u;
      const bool ok = e < ee[q];
      if constexpr (BF) {
        const int j = sci[ok ? e : 0];
        xv[q][u] = X[(int64_t)(ok ? j : 0) * k + c];
      } else {
        xv[q][u] = ok ? X[(int64_t)sci[e] * k + c] : XT(0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < SI; ++q) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = eb[q] + u;
      const bool ok = e < ee[q];
      if constexpr (BF) {
        const TV w = sv[ok ? e : 0];
        a += (double)(ok ? w : TV(0)) * (double)xv[q][u];
      } else {
        if (ok) a += (double)sv[e] * (double)xv[q][u];
      }
    }
    if (ee[q] > eb[q] + CH) a += row_prod_lds<TV, XT>(sci, sv, eb[q] + CH, ee[q], X, k, c);
    out[q] = a;
  }
}

// Block-reduce ND per-lane accumulators (per column) and publish the block's
// partial sums for the finisher.
template <int GK, int ND>
__device__ void block_partials(double (&acc)[ND], const State& S) {
  constexpr int RPB = NT / GK;
  __shared__ double red[ND][NT];
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < ND; ++d) red[d][t] = acc[d];
  __syncthreads();
  if (t < GK) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s = 0.0;
      for (int r = 0; r < RPB; ++r) s += red[d][r * GK + t];
      S.part[((int64_t)d * NBMAX + blockIdx.x) * GK + t] = s;
    }
  }
}

// Grid-stride loop over single rows (streaming kernels).
#define ROW_LOOP                                                                   \
  constexpr int RPB = NT / GK;                                                     \
  const int c = threadIdx.x % GK;                                                  \
  const int rib = threadIdx.x / GK;                                                \
  for (int64_t i = (int64_t)blockIdx.x * RPB + rib; i < n; i += (int64_t)gridDim.x * RPB)

// Tile loop for sparse products: tiles of TR = SUB*RPB rows; every thread of the
// block runs every iteration (the body synchronises).  Workgroups are dispatched
// to the 8 XCDs round-robin (block b on XCD b % 8), and each XCD has its own L2;
// so the tiles are split into 8 contiguous chunks, chunk x processed by the
// blocks of XCD x.  The rows in flight on one XCD then form one window, and
// the gathered rows of X (within the band of the matrix) stay in that XCD's L2.
#define TILE_LOOP                                                                  \
  constexpr int RPB = NT / GK;                                                     \
  constexpr int TR = SUB * RPB;                                                    \
  const int c = threadIdx.x % GK;                                                  \
  const int rib = threadIdx.x / GK;                                                \
  const int64_t ntile_ = (n + TR - 1) / TR;                                        \
  const bool xcd_map_ = xmap && (gridDim.x % 8) == 0;                              \
  const int64_t chunk_ = xcd_map_ ? (ntile_ + 7) / 8 : ntile_;                     \
  const int64_t tfirst_ = xcd_map_ ? (int64_t)(blockIdx.x % 8) * chunk_ : 0;       \
  const int64_t tstep_ = xcd_map_ ? gridDim.x / 8 : gridDim.x;                     \
  const int64_t tlast_ = min<int64_t>(ntile_, tfirst_ + chunk_);                   \
  for (int64_t tile_ = tfirst_ + (xcd_map_ ? blockIdx.x / 8 : blockIdx.x),         \
               t0 = tile_ * TR;                                                    \
       tile_ < tlast_; tile_ += tstep_, t0 = tile_ * TR)

// Stage the entries of rows t0 .. t0+rows-1 in LDS; false when they do not fit.
template <class TV, int CAP>
__device__ __forceinline__ bool stage_tile(const Csr<TV>& A, int64_t t0, int rows, int32_t* s_rp,
                                           int32_t* s_ci, TV* s_v) {
  for (int q = threadIdx.x; q <= rows; q += NT) s_rp[q] = A.rp[t0 + q];
  __syncthreads();
  const int32_t e0 = s_rp[0];
  const int cnt = s_rp[rows] - e0;
  const bool fit = cnt <= CAP;
  if (fit) {
    // the matrix is streamed once per product: non-temporal loads keep it from
    // displacing the gathered rows of X in L2
    for (int q = threadIdx.x; q < cnt; q += NT) {
      s_ci[q] = __builtin_nontemporal_load(&A.ci[e0 + q]);
      s_v[q] = __builtin_nontemporal_load(&A.v[e0 + q]);
    }
  }
  __syncthreads();
  return fit;
}

#define STAGE_DECL(TV, CAP)                   \
  __shared__ int32_t s_rp[SUB * NT / GK + 1]; \
  __shared__ int32_t s_ci[CAP];               \
  __shared__ TV s_v[CAP];

// product of row r (tile-relative) with X; `fit` and `t0` from the tile loop
#define STAGED_PROD(A, X, r)                                                                \
  (fit ? row_prod_lds(s_ci, s_v, s_rp[r] - s_rp[0], s_rp[(r) + 1] - s_rp[0], (X), k, c)    \
       : row_prod((A), t0 + (r), (X), k, c))

// ---- initialisation: x = 0, r = r_hat = rhs, p = v = 0; partial ||r||^2 ----------
template <int GK>
__global__ void __launch_bounds__(NT) k_init(int64_t n, int k, Vec V, State S) {
  double acc[1] = {0.0};
  ROW_LOOP {
    if (c >= k) continue;
    const int64_t q = i * k + c;
    const double b = V.rhs[q];
    V.x[q] = 0.0;
    V.r[q] = b;
    V.rh[q] = b;
    V.p[q] = 0.0;
    V.v[q] = 0.0;
    acc[0] += b * b;
  }
  block_partials<GK, 1>(acc, S);
}

// ---- p = r + beta (p - omega v) (and its FP32 copy) ------------------------------
template <int GK, bool F32>
__global__ void __launch_bounds__(NT) k_pupdate(int64_t n, int k, Vec V, State S) {
  const int cc = threadIdx.x % GK;
  if (!col_on(S, cc, k)) return;
  const double beta = S.beta[cc], omega = S.omega[cc];
  ROW_LOOP {
    const int64_t q = i * k + c;
    const double pv = V.r[q] + beta * (V.p[q] - omega * V.v[q]);
    V.p[q] = pv;
    if constexpr (F32) V.pf[q] = (float)pv;
  }
}

// ---- Y = Op X (plain product for the active columns) -------------------------------
// The lane's SUB rows of the tile are r = sb*RPB + rib; they are handled SI at a
// time with rows_prod_batch (tile staged) or one by one from global memory.
#define TILE_ROWS_PROD(TV, CH, SI, BF, A, X, BODY)                                      \
  if (fit) {                                                                          \
    _Pragma("unroll") for (int b0 = 0; b0 < SUB; b0 += (SI)) {                        \
      int eb[SI], ee[SI];                                                             \
      double out[SI];                                                                 \
      _Pragma("unroll") for (int q = 0; q < (SI); ++q) {                              \
        const int r = (b0 + q) * RPB + rib;                                           \
        eb[q] = r < rows ? s_rp[r] - s_rp[0] : 0;                                     \
        ee[q] = r < rows ? s_rp[r + 1] - s_rp[0] : 0;                                 \
      }                                                                               \
      rows_prod_batch<TV, CH, SI, BF>(s_ci, s_v, eb, ee, (X), k, c, out);              \
      _Pragma("unroll") for (int q = 0; q < (SI); ++q) {                              \
        const int r = (b0 + q) * RPB + rib;                                           \
        if (r < rows) {                                                               \
          const double y = out[q];                                                    \
          const int64_t qq = (t0 + r) * k + c;                                        \
          BODY                                                                        \
        }                                                                             \
      }                                                                               \
    }                                                                                 \
  } else {                                                                            \
    for (int sb = 0; sb < SUB; ++sb) {                                                \
      const int r = sb * RPB + rib;                                                   \
      if (r < rows) {                                                                 \
        const double y = row_prod((A), t0 + r, (X), k, c);                            \
        const int64_t qq = (t0 + r) * k + c;                                          \
        BODY                                                                          \
      }                                                                               \
    }                                                                                 \
  }

template <int GK, class TV, int CH, int SI, int SUBT, class XT>
__global__ void __launch_bounds__(NT) k_spmm(int64_t n, int k, Csr<TV> A, const XT* __restrict__ X,
                                             double* __restrict__ Y, State S, int xmap) {
  constexpr int SUB = SUBT;
  STAGE_DECL(TV, CAP_M)
  const bool on = col_on(S, threadIdx.x % GK, k);
  TILE_LOOP {
    const int rows = (int)min<int64_t>(TR, n - t0);
    const bool fit = stage_tile<TV, CAP_M>(A, t0, rows, s_rp, s_ci, s_v);
    if (on) { TILE_ROWS_PROD(TV, CH, SI, true, A, X, __builtin_nontemporal_store(y, &Y[qq]);) }
    __syncthreads();
  }
}

// ---- v = A p_hat; partial sigma = r_hat^T v --------------------------------------
template <int GK, int SUBT>
__global__ void __launch_bounds__(NT) k_av(int64_t n, int k, Csr<double> A, Vec V, State S, int xmap) {
  constexpr int SUB = SUBT;
  STAGE_DECL(double, CAP_A)
  double acc[1] = {0.0};
  const bool on = col_on(S, threadIdx.x % GK, k);
  TILE_LOOP {
    const int rows = (int)min<int64_t>(TR, n - t0);
    const bool fit = stage_tile<double, CAP_A>(A, t0, rows, s_rp, s_ci, s_v);
    if (on) {
      TILE_ROWS_PROD(double, 8, SUB, false, A, V.ph, __builtin_nontemporal_store(y, &V.v[qq]);
                     acc[0] += __builtin_nontemporal_load(&V.rh[qq]) * y;)
    }
    __syncthreads();
  }
  block_partials<GK, 1>(acc, S);
}

// ---- s = r - alpha v (and its FP32 copy); partial ||s||^2 -------------------------
template <int GK, bool F32>
__global__ void __launch_bounds__(NT) k_s(int64_t n, int k, Vec V, State S) {
  double acc[1] = {0.0};
  const int cc = threadIdx.x % GK;
  const bool on = col_on(S, cc, k);
  const double alpha = on ? S.alpha[cc] : 0.0;
  ROW_LOOP {
    if (!on) break;
    const int64_t q = i * k + c;
    const double sv = V.r[q] - alpha * V.v[q];
    V.s[q] = sv;
    if constexpr (F32) V.sf[q] = (float)sv;
    acc[0] += sv * sv;
  }
  block_partials<GK, 1>(acc, S);
}

// ---- half-step true residual rhs - A (x + alpha p_hat), flagged columns only -------
template <int GK>
__global__ void __launch_bounds__(NT) k_halfcheck(int64_t n, int k, Csr<double> A, Vec V, State S) {
  if (S.any[0] == 0) return;
  double acc[1] = {0.0};
  const int cc = threadIdx.x % GK;
  const bool on = col_on(S, cc, k) && S.half[cc];
  const double al = on ? S.alpha[cc] : 0.0;
  ROW_LOOP {
    if (!on) break;
    double y = 0.0;
    for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int64_t q = (int64_t)A.ci[e] * k + c;
      y += A.v[e] * (V.x[q] + al * V.ph[q]);
    }
    const double rt = V.rhs[i * k + c] - y;
    acc[0] += rt * rt;
  }
  block_partials<GK, 1>(acc, S);
}

// ---- x += alpha p_hat for the columns that converged at the half step -------------
template <int GK>
__global__ void __launch_bounds__(NT) k_halfapply(int64_t n, int k, Vec V, State S) {
  if (S.any[4] == 0) return;
  const int cc = threadIdx.x % GK;
  if (cc >= k || !S.halfconv[cc] || S.status[cc] != ST_ACTIVE) return;
  const double al = S.alpha[cc];
  ROW_LOOP {
    const int64_t q = i * k + c;
    V.x[q] += al * V.ph[q];
  }
}

// ---- t = A s_hat; partials t^T s, t^T t ------------------------------------------
template <int GK, int SUBT>
__global__ void __launch_bounds__(NT) k_at(int64_t n, int k, Csr<double> A, Vec V, State S, int xmap) {
  constexpr int SUB = SUBT;
  STAGE_DECL(double, CAP_A)
  double acc[2] = {0.0, 0.0};
  const int cc = threadIdx.x % GK;
  const bool on = col_on(S, cc, k) && !S.halfconv[cc];
  TILE_LOOP {
    const int rows = (int)min<int64_t>(TR, n - t0);
    const bool fit = stage_tile<double, CAP_A>(A, t0, rows, s_rp, s_ci, s_v);
    if (on) {
      TILE_ROWS_PROD(double, 8, SUB, false, A, V.sh, __builtin_nontemporal_store(y, &V.t[qq]);
                     acc[0] += y * __builtin_nontemporal_load(&V.s[qq]); acc[1] += y * y;)
    }
    __syncthreads();
  }
  block_partials<GK, 2>(acc, S);
}

// ---- x += alpha p_hat + omega s_hat, r = s - omega t; partials r_hat^T r, r^T r -----
template <int GK>
__global__ void __launch_bounds__(NT) k_xr(int64_t n, int k, Vec V, State S) {
  double acc[2] = {0.0, 0.0};
  const int cc = threadIdx.x % GK;
  const bool on = col_on(S, cc, k) && !S.halfconv[cc];
  const double alpha = on ? S.alpha[cc] : 0.0, omega = on ? S.omega[cc] : 0.0;
  ROW_LOOP {
    if (!on) break;
    const int64_t q = i * k + c;
    V.x[q] += alpha * V.ph[q] + omega * V.sh[q];
    const double rv = V.s[q] - omega * V.t[q];
    V.r[q] = rv;
    acc[0] += V.rh[q] * rv;
    acc[1] += rv * rv;
  }
  block_partials<GK, 2>(acc, S);
}

// ---- full-step true residual; partials ||rt||^2, r_hat^T rt; r = rt -----------------
template <int GK>
__global__ void __launch_bounds__(NT) k_fullcheck(int64_t n, int k, Csr<double> A, Vec V, State S) {
  if (S.any[1] == 0) return;
  double acc[2] = {0.0, 0.0};
  const int cc = threadIdx.x % GK;
  const bool on = col_on(S, cc, k) && S.full[cc];
  ROW_LOOP {
    if (!on) break;
    const int64_t q = i * k + c;
    const double rt = V.rhs[q] - row_prod(A, i, V.x, k, c);
    V.r[q] = rt;
    acc[0] += rt * rt;
    acc[1] += V.rh[q] * rt;
  }
  block_partials<GK, 2>(acc, S);
}

// ---- restart: r_hat = r, p = v = 0; partial r^T r ---------------------------------
template <int GK>
__global__ void __launch_bounds__(NT) k_restart(int64_t n, int k, Vec V, State S) {
  if (S.any[2] == 0) return;
  double acc[1] = {0.0};
  const int cc = threadIdx.x % GK;
  const bool on = cc < k && S.rst[cc] && S.status[cc] == ST_ACTIVE;
  ROW_LOOP {
    if (!on) break;
    const int64_t q = i * k + c;
    const double rv = V.r[q];
    V.rh[q] = rv;
    V.p[q] = 0.0;
    V.v[q] = 0.0;
    acc[0] += rv * rv;
  }
  block_partials<GK, 1>(acc, S);
}

// ---- finishers: one block adds the partials and updates the column state -------
enum { F_INIT, F_AV, F_S, F_HALF, F_AT, F_XR, F_FULL, F_RESTART };

constexpr int FNT = 1024;  // finisher threads

template <int GK, int ND, int OP>
__global__ void __launch_bounds__(FNT) k_fin(int k, State S, int nb) {
  constexpr int RPB = FNT / GK;
  __shared__ double red[ND][FNT];
  __shared__ double tot[ND][GK];
  // a finisher whose main kernel returned early (flag not set) has nothing to do
  if (OP == F_HALF && S.any[0] == 0) return;
  if (OP == F_FULL && S.any[1] == 0) return;
  if (OP == F_RESTART && S.any[2] == 0) return;
  const int t = threadIdx.x;
  const int c = t % GK, q = t / GK;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double s0 = 0.0, s1 = 0.0;
    int b = q;
    for (; b + RPB < nb; b += 2 * RPB) {
      s0 += S.part[((int64_t)d * NBMAX + b) * GK + c];
      s1 += S.part[((int64_t)d * NBMAX + b + RPB) * GK + c];
    }
    if (b < nb) s0 += S.part[((int64_t)d * NBMAX + b) * GK + c];
    red[d][t] = s0 + s1;
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
  __syncthreads();
  if (t >= k) return;
  if constexpr (OP == F_INIT) {
    const double rr = tot[0][t];
    S.rho[t] = rr;
    S.rho_old[t] = S.alpha[t] = S.omega[t] = 1.0;
    S.beta[t] = rr;
    S.skip[t] = 0;
    S.restarts[t] = 0;
    S.half[t] = S.full[t] = S.rst[t] = S.halfconv[t] = 0;
    S.iters[t] = 0;
    S.status[t] = (sqrt(rr) < S.thr[t]) ? ST_CONV : ST_ACTIVE;
    if (t == 0) S.any[0] = S.any[1] = S.any[2] = S.any[4] = 0;
  } else if constexpr (OP == F_AV) {
    if (col_on(S, t, k)) {
      const double sig = tot[0][t];
      if (fabs(sig) < TINY) {
        S.skip[t] = 1;
        S.rst[t] = 1;
        S.any[2] = 1;
      } else {
        S.alpha[t] = S.rho[t] / sig;
      }
    }
  } else if constexpr (OP == F_S) {
    if (col_on(S, t, k) && sqrt(tot[0][t]) < S.thr[t]) {
      S.half[t] = 1;
      S.any[0] = 1;
    }
  } else if constexpr (OP == F_HALF) {
    if (col_on(S, t, k) && S.half[t] && sqrt(tot[0][t]) < S.thr[t]) {
      S.halfconv[t] = 1;
      S.any[4] = 1;
    }
  } else if constexpr (OP == F_AT) {
    if (col_on(S, t, k) && !S.halfconv[t]) {
      const double tt = tot[1][t];
      if (tt < TINY) {
        S.skip[t] = 1;
        S.rst[t] = 1;
        S.any[2] = 1;
      } else {
        S.omega[t] = tot[0][t] / tt;
      }
    }
  } else if constexpr (OP == F_XR) {
    if (col_on(S, t, k) && !S.halfconv[t]) {
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
  } else if constexpr (OP == F_FULL) {
    if (col_on(S, t, k) && S.full[t]) {
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
  } else if constexpr (OP == F_RESTART) {
    if (S.rst[t] && S.status[t] == ST_ACTIVE) {
      const double rr = tot[0][t];
      S.rho[t] = rr;
      S.rho_old[t] = S.alpha[t] = S.omega[t] = 1.0;
      S.beta[t] = rr;
      S.restarts[t] += 1;
      if (S.restarts[t] > 1) S.status[t] = ST_BREAK;
    }
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

}  // namespace
}  // namespace sai
