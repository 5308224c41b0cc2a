// Kernels of the batched right-preconditioned BiCGStab (included by krylov.hip).
//
// The vectors of the k systems form n x kp row-major blocks, kp = k rounded up
// to even (the pad column is never active).  A lane owns a pair of columns
// (2l, 2l+1) of one row and moves them with one 16-byte access; LP lanes serve
// a row (LP >= kp/2, from a fixed set so that 64/LP rows fill a wavefront
// well), so a wavefront instruction covers RPW = 64/LP rows.  Compared with
// one lane per column this cuts the number of gather instructions of the
// sparse products, which are bound by the address/data path of the vector
// memory unit rather than by HBM, by about 2.5x for k = 11.
//
// Sparse products stage the column indices and values of a tile of rows (one
// row per lane) in LDS with one coalesced copy, then every lane gathers the
// pairs X[j, 2l..2l+1] of its row in batches whose loads are all issued before
// the first is consumed, sized so that no slot is padded.  Per-column state
// (status, scalars) is read once per kernel.  Dot products are reduced per
// block into partials; a one-block finisher adds the partials in a fixed order
// (deterministic) and updates the per-column scalars and flags.
#pragma once

namespace sai {
namespace {

constexpr int NT = 256;
constexpr int NBMAX = 2048;
constexpr int PSTRIDE = 64;  // most columns per block; partial sums: [ND][NBMAX][kp] doubles
// staged entries per tile (RPB rows): A~ (regular part, about 2p entries per
// row) gets 12 per row, at least 512, at most 2048 (a smaller staging area lets
// more workgroups share a CU); M gets 32 per row, at least 2048, within 40 KB of
// LDS (index and value per entry).  Tiles that do not fit are read from global
// memory.
constexpr int cap_a(int rpb) { return rpb * 12 < 512 ? 512 : (rpb * 12 > 2048 ? 2048 : rpb * 12); }
template <class TV>
constexpr int cap_m(int rpb) {
  const int lim = (40 * 1024) / (int)(4 + sizeof(TV));
  const int want = rpb * 32 < 2048 ? 2048 : rpb * 32;
  return want < lim ? want : lim;
}
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
  int* pend;  // t^T t below TINY at a column that awaits its half-step check
  int* any;   // 0 half, 1 full, 2 restart, 3 active count, 4 half-converged
  double* part;
  int nt;     // output blocks stored non-temporally (st2)
  int ntl;    // streamed (not gathered) block reads non-temporal (lds2)
};

// n x kp blocks (b: the right-hand sides, copied in with the pad column zeroed)
struct Vec {
  double *b, *x, *r, *rh, *p, *v, *s, *ph, *sh, *t;
};

__device__ __forceinline__ bool col_on(const State& S, int c, int k) {
  return c < k && S.status[c] == ST_ACTIVE && S.skip[c] == 0;
}

__device__ __forceinline__ double2 ld2(const double* __restrict__ p, int64_t q) {
  return *reinterpret_cast<const double2*>(p + q);
}
// a streamed read of a block (the row's own pair, not a gathered one); with ntl
// non-temporal, which leaves L2 to the gathered rows
__device__ __forceinline__ double2 lds2(const double* __restrict__ p, int64_t q, int ntl) {
  typedef double d2v_ __attribute__((ext_vector_type(2)));
  if (ntl) {
    const d2v_ v = __builtin_nontemporal_load(reinterpret_cast<const d2v_*>(p + q));
    return make_double2(v.x, v.y);
  }
  return *reinterpret_cast<const double2*>(p + q);
}

// store the pair (a, b) at q, q+1, each half only where its column is on; with
// pad (the second column is the block's pad column, c0 + 1 = k) as one 16-byte
// store when the first is on.  The pad column is zero in every block and each
// kernel computes zero for it from zero inputs (its scalars are zero), so the
// store leaves it unchanged; a single 16-byte store instead of a divergent pair
// of stores made the M product on the 52-wide block about 10% faster.  With nt
// (blocks larger than the L2s together; State::nt) the stores are non-temporal:
// an output block is next read by another kernel, and keeping it out of the
// caches' recently-used lines leaves them to the rows the sparse products gather
// (every kernel of the iteration 3-7% faster at 160^3); blocks that fit the L2s
// are read back from there.
typedef double sai_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st2(double* __restrict__ p, int64_t q, double a, double b, bool o0,
                                    bool o1, bool pad, int nt) {
  if (o0 && (o1 || pad)) {
    const sai_d2v v = {a, b};
    if (nt) __builtin_nontemporal_store(v, reinterpret_cast<sai_d2v*>(p + q));
    else *reinterpret_cast<sai_d2v*>(p + q) = v;
  } else if (nt) {
    if (o0) __builtin_nontemporal_store(a, p + q);
    if (o1) __builtin_nontemporal_store(b, p + q + 1);
  } else {
    if (o0) p[q] = a;
    if (o1) p[q + 1] = b;
  }
}

// Lane geometry: LP lanes per row, RPW rows per wavefront, RPB rows per block.
#define LANES(LP)                                                              \
  constexpr int RPW = 64 / (LP);                                               \
  constexpr int RPB = RPW * (NT / 64);                                         \
  const int l_ = (int)(threadIdx.x & 63) % (LP);                               \
  const bool lok_ = ((int)(threadIdx.x & 63) / (LP)) < RPW;                    \
  const int rib = (int)(threadIdx.x >> 6) * RPW + (int)(threadIdx.x & 63) / (LP); \
  const int c0 = 2 * l_;                                                       \
  const bool live = lok_ && c0 < k;                                            \
  const bool pad1_ = c0 + 1 == k;                                              \
  (void)RPB;                                                                   \
  (void)live;                                                                  \
  (void)pad1_;

// rows i handled by this lane in a grid-stride loop (streaming kernels)
#define ROW_LOOP for (int64_t i = (int64_t)blockIdx.x * RPB + rib; i < n; i += (int64_t)gridDim.x * RPB)

// Product of one row (entries e..ee of (ci, v)) with the column pair c0, c0+1
// of X (row stride kp): batches of CH entries while at least CH remain (all
// loads of a batch issued before the first is consumed), then one batch of CH2,
// then single entries, so that no load slot is wasted on a padded entry (the
// gathers are bound by the vector memory unit's instruction throughput).
template <class TV, int CH, int CH2>
__device__ __forceinline__ void row_prod(const int32_t* __restrict__ ci, const TV* __restrict__ v, int e,
                                         int ee, const double* __restrict__ X, int kp, int c0, double& a0,
                                         double& a1) {
  a0 = a1 = 0.0;
  for (; e + CH <= ee; e += CH) {
    double2 xv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) xv[u] = ld2(X, (int64_t)ci[e + u] * kp + c0);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const double w = (double)v[e + u];
      a0 += w * xv[u].x;
      a1 += w * xv[u].y;
    }
  }
  if (CH2 > 0 && e + CH2 <= ee) {
    double2 xv[CH2 > 0 ? CH2 : 1];
#pragma unroll
    for (int u = 0; u < CH2; ++u) xv[u] = ld2(X, (int64_t)ci[e + u] * kp + c0);
#pragma unroll
    for (int u = 0; u < CH2; ++u) {
      const double w = (double)v[e + u];
      a0 += w * xv[u].x;
      a1 += w * xv[u].y;
    }
    e += CH2;
  }
  for (; e < ee; ++e) {
    const double2 x = ld2(X, (int64_t)ci[e] * kp + c0);
    const double w = (double)v[e];
    a0 += w * x.x;
    a1 += w * x.y;
  }
}

// Product of one row with X + al P (column pair c0, c0+1; al per column), each
// entry added as v (x + al p) in order, the loads batched as in row_prod.
template <class TV, int CH, int CH2>
__device__ __forceinline__ void row_prod_xp(const int32_t* __restrict__ ci, const TV* __restrict__ v, int e,
                                            int ee, const double* __restrict__ X,
                                            const double* __restrict__ P, double al0, double al1, int kp,
                                            int c0, double& a0, double& a1) {
  a0 = a1 = 0.0;
  for (; e + CH <= ee; e += CH) {
    double2 xv[CH], pv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int64_t q = (int64_t)ci[e + u] * kp + c0;
      xv[u] = ld2(X, q);
      pv[u] = ld2(P, q);
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const double w = (double)v[e + u];
      a0 += w * (xv[u].x + al0 * pv[u].x);
      a1 += w * (xv[u].y + al1 * pv[u].y);
    }
  }
  if (CH2 > 0 && e + CH2 <= ee) {
    double2 xv[CH2 > 0 ? CH2 : 1], pv[CH2 > 0 ? CH2 : 1];
#pragma unroll
    for (int u = 0; u < CH2; ++u) {
      const int64_t q = (int64_t)ci[e + u] * kp + c0;
      xv[u] = ld2(X, q);
      pv[u] = ld2(P, q);
    }
#pragma unroll
    for (int u = 0; u < CH2; ++u) {
      const double w = (double)v[e + u];
      a0 += w * (xv[u].x + al0 * pv[u].x);
      a1 += w * (xv[u].y + al1 * pv[u].y);
    }
    e += CH2;
  }
  for (; e < ee; ++e) {
    const int64_t q = (int64_t)ci[e] * kp + c0;
    const double2 x = ld2(X, q), p = ld2(P, q);
    const double w = (double)v[e];
    a0 += w * (x.x + al0 * p.x);
    a1 += w * (x.y + al1 * p.y);
  }
}

// Block-reduce ND per-lane accumulator pairs (per column) in a fixed order and
// publish the block's partial sums for the finisher.  Slot 2t+j (of 2 NT) holds
// thread t's value for column 2((t & 63) % LP) + j, so slot s belongs to wave
// s / 128 and wave row (s % 128) / (2 LP).  A tree first adds the wavefronts
// (strides 256, 128), then, while LP is a power of two, the rows of a wavefront
// (strides 64 ... 2 LP); for LP = 6 and 12 a short serial sum over the 64 / LP
// rows finishes.
template <int LP, int ND>
__device__ void block_partials(double (&acc)[ND][2], const State& S, int kp) {
  constexpr int RPW = 64 / LP;
  constexpr bool POW2 = (LP & (LP - 1)) == 0;
  __shared__ double red[ND][2 * NT];
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    red[d][2 * t] = acc[d][0];
    red[d][2 * t + 1] = acc[d][1];
  }
  __syncthreads();
  // across wavefronts, then (power-of-two LP) across the rows of a wavefront
  constexpr int LAST = POW2 ? 2 * LP : 128;
#pragma unroll 1
  for (int stride = NT; stride >= LAST; stride >>= 1) {
    if (t < stride) {
#pragma unroll
      for (int d = 0; d < ND; ++d) red[d][t] += red[d][t + stride];
    }
    __syncthreads();
  }
  if (t < kp) {
#pragma unroll 1
    for (int d = 0; d < ND; ++d) {
      double s = red[d][t];
      if constexpr (!POW2) {
#pragma unroll 1
        for (int rw = 1; rw < RPW; ++rw) s += red[d][t + 2 * LP * rw];
      }
      S.part[((int64_t)d * NBMAX + blockIdx.x) * kp + t] = s;
    }
  }
}

// Tile loop for sparse products: tiles of TR = RPB rows (one per lane); every thread of
// the block runs every iteration (the body synchronises).  Workgroups are
// dispatched to the 8 XCDs round-robin (block b on XCD b % 8), and each XCD
// has its own L2.  xmap selects which tiles an XCD's blocks take:
//   0   round-robin over all tiles (consecutive tiles on different XCDs);
//   1   8 contiguous chunks of the tiles, chunk x on XCD x (the band of
//       gathered rows of X stays in that XCD's L2; for blocks that fit the MALL);
//   C>1 blocked interleave: super-chunks of 8 C consecutive tiles, whose x-th
//       run of C tiles goes to XCD x.  The XCDs advance through the rows
//       together (one shared window of gathered rows in the MALL) while each
//       keeps a contiguous run of rows, whose nearby gathers hit its L2.
// Tile m of an XCD (m = b, b + G, ... for its b-th of G blocks) is
// (m / C) 8 C + x C + m % C, increasing in m.
//
// The block's position m = q C + r advances by G per tile without a division in
// the loop (the 64-bit divisions it took otherwise cost about a tenth of the M
// product's time); tile counts fit in 32 bits (row indices are 32-bit).
#define TILE_LOOP                                                                     \
  constexpr int TR = RPB;                                                             \
  const int ntile_ = (int)((n + TR - 1) / TR);                                        \
  const int xm_ = (gridDim.x % 8) == 0 ? xmap : 0;                                    \
  const int G_ = xm_ ? (int)gridDim.x / 8 : (int)gridDim.x;                           \
  const int b_ = xm_ ? (int)blockIdx.x / 8 : (int)blockIdx.x;                         \
  const int x_ = (int)blockIdx.x % 8;                                                 \
  const int C_ = xm_ == 1 ? (ntile_ + 7) / 8 : (xm_ > 1 ? xm_ : 1);                   \
  const int Gq_ = G_ / C_, Gr_ = G_ % C_;                                             \
  int q_ = b_ / C_, r_ = b_ % C_;                                                     \
  int tile_ = xm_ ? q_ * 8 * C_ + x_ * C_ + r_ : q_;                                  \
  for (int64_t t0 = (int64_t)tile_ * TR; tile_ < ntile_;                              \
       r_ += Gr_, q_ += Gq_ + (r_ >= C_ ? 1 : 0), r_ -= (r_ >= C_ ? C_ : 0),          \
       tile_ = xm_ ? q_ * 8 * C_ + x_ * C_ + r_ : q_, t0 = (int64_t)tile_ * TR)

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
    // displacing the gathered rows of X in L2.  Each thread issues up to SU
    // rounds of loads before its first store, so that staging a tile of many
    // entries waits on memory once per SU rounds, not once per round.
    constexpr int SU = 8;
    for (int q0 = threadIdx.x; q0 < cnt; q0 += SU * NT) {
      int32_t c[SU];
      TV v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int q = q0 + u * NT;
        c[u] = q < cnt ? __builtin_nontemporal_load(&A.ci[e0 + q]) : 0;
        v[u] = q < cnt ? __builtin_nontemporal_load(&A.v[e0 + q]) : TV(0);
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int q = q0 + u * NT;
        if (q < cnt) {
          s_ci[q] = c[u];
          s_v[q] = v[u];
        }
      }
    }
  }
  __syncthreads();
  return fit;
}

#define STAGE_DECL(TV, CAP, TRW)       \
  __shared__ int32_t s_rp[(TRW) + 1]; \
  __shared__ int32_t s_ci[CAP];       \
  __shared__ TV s_v[CAP];

// The lane's row of the tile is r = rib (from LDS when the tile was staged,
// else from the matrix in global memory).  If r < rows: PRE (loads issued
// before the gathers), then BODY with y0, y1 (the pair's products) and qq (the
// index of the pair's first element).
#define TILE_ROW_PROD(TV, CH, CH2, A, X, PRE, BODY)                                     \
  if (rib < rows) {                                                                     \
    const int64_t qq = (t0 + rib) * kp + c0;                                            \
    PRE                                                                                 \
    double y0, y1;                                                                      \
    if (fit)                                                                            \
      row_prod<TV, CH, CH2>(s_ci, s_v, s_rp[rib] - s_rp[0], s_rp[rib + 1] - s_rp[0], (X), \
                            kp, c0, y0, y1);                                            \
    else                                                                                \
      row_prod<TV, CH, CH2>((A).ci, (A).v, s_rp[rib], s_rp[rib + 1], (X), kp, c0, y0, y1); \
    BODY                                                                                \
  }

// The same without LDS staging (STG = false): the lane's row t0 + rib is read
// from the matrix in global memory (the lanes of a row load the same entries,
// served by one access; non-temporal loads here were slower), and the tile
// loop needs no workgroup barrier.  For short rows and narrow blocks the
// staging's barriers and dependent loads cost more than they save.
#define GLOBAL_ROW_PROD(TV, CH, CH2, A, X, PRE, BODY)                                   \
  if (rib < rows) {                                                                     \
    const int64_t i_ = t0 + rib;                                                        \
    const int64_t qq = i_ * kp + c0;                                                    \
    PRE                                                                                 \
    double y0, y1;                                                                      \
    row_prod<TV, CH, CH2>((A).ci, (A).v, (A).rp[i_], (A).rp[i_ + 1], (X), kp, c0, y0, y1); \
    BODY                                                                                \
  }

// ---- initialisation: b = R (pad column 0), x = 0, r = r_hat = b, p = v = 0 -------
template <int LP>
__global__ void __launch_bounds__(NT) k_init(int64_t n, int k, int kp, const double* __restrict__ R,
                                             Vec V, State S) {
  LANES(LP)
  double acc[1][2] = {{0.0, 0.0}};
  if (lok_ && c0 < kp) {
    ROW_LOOP {
      const int64_t q = i * kp + c0;
      const double b0 = R[i * k + c0];
      const double b1 = c0 + 1 < k ? R[i * k + c0 + 1] : 0.0;
      const double2 bb = make_double2(b0, b1), zz = make_double2(0.0, 0.0);
      *reinterpret_cast<double2*>(V.b + q) = bb;
      *reinterpret_cast<double2*>(V.x + q) = zz;
      *reinterpret_cast<double2*>(V.r + q) = bb;
      *reinterpret_cast<double2*>(V.rh + q) = bb;
      *reinterpret_cast<double2*>(V.p + q) = zz;
      *reinterpret_cast<double2*>(V.v + q) = zz;
      if (c0 + 1 == k) {  // zero the pad column of the other blocks
        V.s[q + 1] = V.ph[q + 1] = V.sh[q + 1] = V.t[q + 1] = 0.0;
      }
      acc[0][0] += b0 * b0;
      acc[0][1] += b1 * b1;
    }
  }
  block_partials<LP, 1>(acc, S, kp);
}

// ---- p = r + beta (p - omega v) -------------------------------------------------
template <int LP>
__global__ void __launch_bounds__(NT) k_pupdate(int64_t n, int k, int kp, Vec V, State S) {
  LANES(LP)
  const bool o0 = lok_ && col_on(S, c0, k), o1 = lok_ && col_on(S, c0 + 1, k);
  if (!o0 && !o1) return;
  const double be0 = o0 ? S.beta[c0] : 0.0, om0 = o0 ? S.omega[c0] : 0.0;
  const double be1 = o1 ? S.beta[c0 + 1] : 0.0, om1 = o1 ? S.omega[c0 + 1] : 0.0;
  ROW_LOOP {
    const int64_t q = i * kp + c0;
    const double2 r = lds2(V.r, q, S.ntl), p = lds2(V.p, q, S.ntl), v = lds2(V.v, q, S.ntl);
    st2(V.p, q, r.x + be0 * (p.x - om0 * v.x), r.y + be1 * (p.y - om1 * v.y), o0, o1, pad1_, S.nt);
  }
}

// ---- Y = Op X (plain product for the active columns) -------------------------------
template <int LP, class TV, int CH, int CH2>
__global__ void __launch_bounds__(NT) k_spmm(int64_t n, int k, int kp, Csr<TV> A,
                                             const double* __restrict__ X, double* __restrict__ Y,
                                             State S, int xmap) {
  LANES(LP)
  constexpr int CAP_M = cap_m<TV>(RPB);
  STAGE_DECL(TV, CAP_M, RPB)
  if (S.any[3] == 0) return;
  const bool o0 = lok_ && col_on(S, c0, k), o1 = lok_ && col_on(S, c0 + 1, k);
  TILE_LOOP {
    const int rows = (int)min<int64_t>(TR, n - t0);
    const bool fit = stage_tile<TV, CAP_M>(A, t0, rows, s_rp, s_ci, s_v);
    if (o0 || o1) { TILE_ROW_PROD(TV, CH, CH2, A, X, , st2(Y, qq, y0, y1, o0, o1, pad1_, S.nt);) }
    __syncthreads();
  }
}

// ---- v = A p_hat; partial sigma = r_hat^T v --------------------------------------
template <int LP, int CH, int CH2, bool STG = true>
__global__ void __launch_bounds__(NT) k_av(int64_t n, int k, int kp, Csr<double> A, Vec V, State S,
                                           int xmap) {
  LANES(LP)
  double acc[1][2] = {{0.0, 0.0}};
  const bool o0 = lok_ && col_on(S, c0, k), o1 = lok_ && col_on(S, c0 + 1, k);
  if constexpr (STG) {
    constexpr int CAP_A = cap_a(RPB);
    STAGE_DECL(double, CAP_A, RPB)
    if (S.any[3] != 0) {
      TILE_LOOP {
        const int rows = (int)min<int64_t>(TR, n - t0);
        const bool fit = stage_tile<double, CAP_A>(A, t0, rows, s_rp, s_ci, s_v);
        if (o0 || o1) {
          TILE_ROW_PROD(double, CH, CH2, A, V.ph, const double2 rh = lds2(V.rh, qq, S.ntl);,
                        st2(V.v, qq, y0, y1, o0, o1, pad1_, S.nt);
                        if (o0) acc[0][0] += rh.x * y0; if (o1) acc[0][1] += rh.y * y1;)
        }
        __syncthreads();
      }
    }
  } else {
    if (S.any[3] != 0 && (o0 || o1)) {
      TILE_LOOP {
        const int rows = (int)min<int64_t>(TR, n - t0);
        GLOBAL_ROW_PROD(double, CH, CH2, A, V.ph, const double2 rh = lds2(V.rh, qq, S.ntl);,
                        st2(V.v, qq, y0, y1, o0, o1, pad1_, S.nt);
                        if (o0) acc[0][0] += rh.x * y0; if (o1) acc[0][1] += rh.y * y1;)
      }
    }
  }
  block_partials<LP, 1>(acc, S, kp);
}

// ---- s = r - alpha v (its norm is summed by k_at) --------------------------------
template <int LP>
__global__ void __launch_bounds__(NT) k_s(int64_t n, int k, int kp, Vec V, State S) {
  LANES(LP)
  const bool o0 = lok_ && col_on(S, c0, k), o1 = lok_ && col_on(S, c0 + 1, k);
  if (!o0 && !o1) return;
  const double al0 = o0 ? S.alpha[c0] : 0.0, al1 = o1 ? S.alpha[c0 + 1] : 0.0;
  ROW_LOOP {
    const int64_t q = i * kp + c0;
    const double2 r = lds2(V.r, q, S.ntl), v = lds2(V.v, q, S.ntl);
    st2(V.s, q, r.x - al0 * v.x, r.y - al1 * v.y, o0, o1, pad1_, S.nt);
  }
}

// ---- half-step true residual b - A (x + alpha p_hat), flagged columns only -------
// (persistent grid over tiles, A~ staged in LDS; called with the A~ products' grid)
template <int LP>
__global__ void __launch_bounds__(NT) k_halfcheck(int64_t n, int k, int kp, Csr<double> A, Vec V,
                                                  State S, int xmap) {
  if (S.any[0] == 0) return;
  LANES(LP)
  constexpr int CAP_A = cap_a(RPB);
  STAGE_DECL(double, CAP_A, RPB)
  double acc[1][2] = {{0.0, 0.0}};
  const bool o0 = lok_ && col_on(S, c0, k) && S.half[c0];
  const bool o1 = lok_ && col_on(S, c0 + 1, k) && S.half[c0 + 1];
  const double al0 = o0 ? S.alpha[c0] : 0.0, al1 = o1 ? S.alpha[c0 + 1] : 0.0;
  TILE_LOOP {
    const int rows = (int)min<int64_t>(TR, n - t0);
    const bool fit = stage_tile<double, CAP_A>(A, t0, rows, s_rp, s_ci, s_v);
    if ((o0 || o1) && rib < rows) {
      const int64_t qq = (t0 + rib) * kp + c0;
      double y0, y1;
      if (fit)
        row_prod_xp<double, 4, 2>(s_ci, s_v, s_rp[rib] - s_rp[0], s_rp[rib + 1] - s_rp[0], V.x, V.ph, al0,
                                  al1, kp, c0, y0, y1);
      else
        row_prod_xp<double, 4, 2>(A.ci, A.v, s_rp[rib], s_rp[rib + 1], V.x, V.ph, al0, al1, kp, c0, y0, y1);
      const double2 b = lds2(V.b, qq, S.ntl);
      const double r0 = b.x - y0, r1 = b.y - y1;
      if (o0) acc[0][0] += r0 * r0;
      if (o1) acc[0][1] += r1 * r1;
    }
    __syncthreads();
  }
  block_partials<LP, 1>(acc, S, kp);
}

// ---- t = A s_hat; partials t^T s, t^T t, s^T s ------------------------------------
template <int LP, int CH, int CH2, bool STG = true>
__global__ void __launch_bounds__(NT) k_at(int64_t n, int k, int kp, Csr<double> A, Vec V, State S,
                                           int xmap) {
  LANES(LP)
  double acc[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  const bool o0 = lok_ && col_on(S, c0, k), o1 = lok_ && col_on(S, c0 + 1, k);
#define AT_BODY                                                                                  \
  st2(V.t, qq, y0, y1, o0, o1, pad1_, S.nt);                                                                  \
  if (o0) { acc[0][0] += y0 * sv.x; acc[1][0] += y0 * y0; acc[2][0] += sv.x * sv.x; }            \
  if (o1) { acc[0][1] += y1 * sv.y; acc[1][1] += y1 * y1; acc[2][1] += sv.y * sv.y; }
  if constexpr (STG) {
    constexpr int CAP_A = cap_a(RPB);
    STAGE_DECL(double, CAP_A, RPB)
    if (S.any[3] != 0) {
      TILE_LOOP {
        const int rows = (int)min<int64_t>(TR, n - t0);
        const bool fit = stage_tile<double, CAP_A>(A, t0, rows, s_rp, s_ci, s_v);
        if (o0 || o1) { TILE_ROW_PROD(double, CH, CH2, A, V.sh, const double2 sv = lds2(V.s, qq, S.ntl);, AT_BODY) }
        __syncthreads();
      }
    }
  } else {
    if (S.any[3] != 0 && (o0 || o1)) {
      TILE_LOOP {
        const int rows = (int)min<int64_t>(TR, n - t0);
        GLOBAL_ROW_PROD(double, CH, CH2, A, V.sh, const double2 sv = lds2(V.s, qq, S.ntl);, AT_BODY)
      }
    }
  }
#undef AT_BODY
  block_partials<LP, 3>(acc, S, kp);
}

// ---- x += alpha p_hat + omega s_hat, r = s - omega t; partials r_hat^T r, r^T r -----
// Columns that converged at the half step only take x += alpha p_hat.
template <int LP>
__global__ void __launch_bounds__(NT) k_xr(int64_t n, int k, int kp, Vec V, State S) {
  LANES(LP)
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  const bool a0 = lok_ && col_on(S, c0, k), a1 = lok_ && col_on(S, c0 + 1, k);
  const bool h0 = a0 && S.halfconv[c0], h1 = a1 && S.halfconv[c0 + 1];
  const bool o0 = a0 && !h0, o1 = a1 && !h1;  // full updates
  const double al0 = a0 ? S.alpha[c0] : 0.0, om0 = o0 ? S.omega[c0] : 0.0;
  const double al1 = a1 ? S.alpha[c0 + 1] : 0.0, om1 = o1 ? S.omega[c0 + 1] : 0.0;
  if (a0 || a1) {
    ROW_LOOP {
      const int64_t q = i * kp + c0;
      const double2 x = lds2(V.x, q, S.ntl), ph = lds2(V.ph, q, S.ntl), sh = lds2(V.sh, q, S.ntl);
      st2(V.x, q, x.x + al0 * ph.x + om0 * sh.x, x.y + al1 * ph.y + om1 * sh.y, a0, a1, pad1_, S.nt);
      if (o0 || o1) {
        const double2 s = lds2(V.s, q, S.ntl), t = lds2(V.t, q, S.ntl), rh = lds2(V.rh, q, S.ntl);
        const double r0 = s.x - om0 * t.x, r1 = s.y - om1 * t.y;
        st2(V.r, q, r0, r1, o0, o1, pad1_, S.nt);
        if (o0) { acc[0][0] += rh.x * r0; acc[1][0] += r0 * r0; }
        if (o1) { acc[0][1] += rh.y * r1; acc[1][1] += r1 * r1; }
      }
    }
  }
  block_partials<LP, 2>(acc, S, kp);
}

// ---- full-step true residual; partials ||rt||^2, r_hat^T rt; r = rt -----------------
// (persistent grid over tiles, A~ staged in LDS; called with the A~ products' grid)
template <int LP>
__global__ void __launch_bounds__(NT) k_fullcheck(int64_t n, int k, int kp, Csr<double> A, Vec V,
                                                  State S, int xmap) {
  if (S.any[1] == 0) return;
  LANES(LP)
  constexpr int CAP_A = cap_a(RPB);
  STAGE_DECL(double, CAP_A, RPB)
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  const bool o0 = lok_ && col_on(S, c0, k) && S.full[c0];
  const bool o1 = lok_ && col_on(S, c0 + 1, k) && S.full[c0 + 1];
  TILE_LOOP {
    const int rows = (int)min<int64_t>(TR, n - t0);
    const bool fit = stage_tile<double, CAP_A>(A, t0, rows, s_rp, s_ci, s_v);
    if (o0 || o1) {
      TILE_ROW_PROD(double, 4, 2, A, V.x, const double2 b = lds2(V.b, qq, S.ntl); const double2 rh = lds2(V.rh, qq, S.ntl);,
                    const double r0 = b.x - y0; const double r1 = b.y - y1;
                    st2(V.r, qq, r0, r1, o0, o1, pad1_, S.nt);
                    if (o0) { acc[0][0] += r0 * r0; acc[1][0] += rh.x * r0; }
                    if (o1) { acc[0][1] += r1 * r1; acc[1][1] += rh.y * r1; })
    }
    __syncthreads();
  }
  block_partials<LP, 2>(acc, S, kp);
}

// ---- restart: r_hat = r, p = v = 0; partial r^T r ---------------------------------
template <int LP>
__global__ void __launch_bounds__(NT) k_restart(int64_t n, int k, int kp, Vec V, State S) {
  if (S.any[2] == 0) return;
  LANES(LP)
  double acc[1][2] = {{0.0, 0.0}};
  const bool o0 = lok_ && c0 < k && S.rst[c0] && S.status[c0] == ST_ACTIVE;
  const bool o1 = lok_ && c0 + 1 < k && S.rst[c0 + 1] && S.status[c0 + 1] == ST_ACTIVE;
  if (o0 || o1) {
    ROW_LOOP {
      const int64_t q = i * kp + c0;
      const double2 r = lds2(V.r, q, S.ntl);
      st2(V.rh, q, r.x, r.y, o0, o1, pad1_, S.nt);
      st2(V.p, q, 0.0, 0.0, o0, o1, pad1_, S.nt);
      st2(V.v, q, 0.0, 0.0, o0, o1, pad1_, S.nt);
      if (o0) acc[0][0] += r.x * r.x;
      if (o1) acc[0][1] += r.y * r.y;
    }
  }
  block_partials<LP, 1>(acc, S, kp);
}

// ---- the solution block X (n x k, the caller's) from x (n x kp) -------------------
template <int LP>
__global__ void __launch_bounds__(NT) k_copy_out(int64_t n, int k, int kp, const double* __restrict__ x,
                                                 double* __restrict__ X) {
  LANES(LP)
  if (!live) return;
  ROW_LOOP {
    const double2 v = ld2(x, i * kp + c0);
    X[i * k + c0] = v.x;
    if (c0 + 1 < k) X[i * k + c0 + 1] = v.y;
  }
}

// ---- end of an iteration: record iterations, clear flags, count active columns ----
// (all threads of the block call it; it synchronises)
__device__ void iter_end_body(int k, const State& S, int it, int maxit) {
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
    S.half[t] = S.full[t] = S.rst[t] = S.halfconv[t] = S.pend[t] = 0;
    if (st == ST_ACTIVE) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (t == 0) {
    S.any[0] = S.any[1] = S.any[2] = S.any[4] = 0;
    S.any[3] = cnt;
  }
}

// ---- finishers: one block adds the partials and updates the column state -------
enum { F_INIT, F_AV, F_AT, F_HALF, F_XR, F_FULL, F_RESTART_END };

constexpr int FNT = 1024;  // finisher threads

template <int ND, int OP>
// force_it, force_it2 (the F_XR and F_FULL finishers): at the end of iteration
// it == force_it (or force_it2) every active column that has not converged is
// handled as a breakdown (restart), so that the restart path and the second
// breakdown can be tested on well-conditioned systems; 0 (the default) never
// matches.
__global__ void __launch_bounds__(FNT) k_fin(int k, State S, int nb, int it = 0, int maxit = 0,
                                             int force_it = 0, int force_it2 = 0) {
  const bool forced = it > 0 && (it == force_it || it == force_it2);
  // partial sums are read as column pairs; U independent sums per pair and d
  // keep U loads of every d in flight (the partials come from every XCD, so
  // each round of loads is a trip past the L2)
  constexpr int U = ND == 1 ? 16 : 8;
  __shared__ double2 red[ND][FNT];
  __shared__ double tot[ND][PSTRIDE];
  // a finisher whose main kernel returned early (flag not set) has nothing to do
  if (OP == F_HALF && S.any[0] == 0) return;
  if (OP == F_FULL && S.any[1] == 0) return;
  // (F_RESTART_END always runs: it also closes the iteration)
  // thread t sums the partials b = q, q + fq, ... of the column pair c2 = t % kh
  // (columns 2 c2, 2 c2 + 1; fq threads per pair)
  const int t = threadIdx.x;
  const int kh = (k + 1) >> 1;
  const int fq = FNT / kh;
  const int c2 = t % kh, q = t / kh;
  const bool sum = OP != F_RESTART_END || S.any[2] != 0;
  // the column state each update reads, loaded now so that these loads overlap
  // the partial sums' (nothing below writes a field before reading it)
  int st_status = 0, st_skip = 0, st_flag = 0, st_pend = 0, st_restarts = 0;
  double st_rho = 0.0, st_rho_old = 0.0, st_alpha = 0.0, st_omega = 0.0, st_thr = 0.0;
  if (t < k) {
    st_status = S.status[t];
    st_skip = S.skip[t];
    if constexpr (OP == F_INIT || OP == F_AT || OP == F_HALF || OP == F_XR || OP == F_FULL) st_thr = S.thr[t];
    if constexpr (OP == F_AV || OP == F_XR) st_rho = S.rho[t];
    if constexpr (OP == F_XR || OP == F_FULL) {
      st_alpha = S.alpha[t];
      st_omega = S.omega[t];
    }
    if constexpr (OP == F_FULL) st_rho_old = S.rho_old[t];
    if constexpr (OP == F_HALF) {
      st_flag = S.half[t];
      st_pend = S.pend[t];
    }
    if constexpr (OP == F_XR) st_flag = S.halfconv[t];
    if constexpr (OP == F_FULL) st_flag = S.full[t];
    if constexpr (OP == F_RESTART_END) {
      st_flag = S.rst[t];
      st_restarts = S.restarts[t];
    }
  }
  const bool on = t < k && st_status == ST_ACTIVE && st_skip == 0;  // col_on(S, t, k)
  double2 acc[ND][U];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int u = 0; u < U; ++u) acc[d][u] = make_double2(0.0, 0.0);
  if (sum && q < fq) {
    const double* P = S.part + 2 * c2;
#pragma unroll 1
    for (int b = q; b < nb; b += U * fq) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int bb = b + u * fq;
        if (bb < nb) {
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            const double2 v = *(const double2*)(P + ((int64_t)d * NBMAX + bb) * (2 * kh));
            acc[d][u].x += v.x;
            acc[d][u].y += v.y;
          }
        }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
#pragma unroll
    for (int w = U / 2; w >= 1; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u) {
        acc[d][u].x += acc[d][u + w].x;
        acc[d][u].y += acc[d][u + w].y;
      }
    red[d][t] = acc[d][0];
  }
  __syncthreads();
  // the fq sums of a pair meet in a tree: at each level the upper half of the
  // remaining sums (q >= h) is added onto the lower half (q - h)
#pragma unroll 1
  for (int cur = fq; cur > 1;) {
    const int h = (cur + 1) >> 1;
    if (q + h < cur) {
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const double2 o = red[d][t + h * kh];
        red[d][t].x += o.x;
        red[d][t].y += o.y;
      }
    }
    __syncthreads();
    cur = h;
  }
  if (t < k) {
#pragma unroll
    for (int d = 0; d < ND; ++d) tot[d][t] = (t & 1) ? red[d][t >> 1].y : red[d][t >> 1].x;
  }
  __syncthreads();
  if (t >= k) {
    if constexpr (OP == F_RESTART_END) iter_end_body(k, S, it, maxit);
    return;
  }
  if constexpr (OP == F_INIT) {
    const double rr = tot[0][t];
    S.rho[t] = rr;
    S.rho_old[t] = S.alpha[t] = S.omega[t] = 1.0;
    S.beta[t] = rr;
    S.skip[t] = 0;
    S.restarts[t] = 0;
    S.half[t] = S.full[t] = S.rst[t] = S.halfconv[t] = S.pend[t] = 0;
    S.iters[t] = 0;
    S.status[t] = (sqrt(rr) < st_thr) ? ST_CONV : ST_ACTIVE;
    if (t == 0) S.any[0] = S.any[1] = S.any[2] = S.any[4] = 0;
  } else if constexpr (OP == F_AV) {
    if (on) {
      const double sig = tot[0][t];
      if (fabs(sig) < TINY) {
        S.skip[t] = 1;
        S.rst[t] = 1;
        S.any[2] = 1;
      } else {
        S.alpha[t] = st_rho / sig;
      }
    }
  } else if constexpr (OP == F_AT) {
    // partials: t^T s, t^T t, s^T s.  The half-step check (||s|| < thr) is flagged
    // here; a column waiting for it keeps a tiny t^T t as pending (a breakdown only
    // if the check fails: s ~ 0 makes t ~ 0)
    if (on) {
      const double tt = tot[1][t];
      const bool half = sqrt(tot[2][t]) < st_thr;
      if (half) {
        S.half[t] = 1;
        S.any[0] = 1;
      }
      if (tt < TINY) {
        if (half) {
          S.pend[t] = 1;
        } else {
          S.skip[t] = 1;
          S.rst[t] = 1;
          S.any[2] = 1;
        }
      } else {
        S.omega[t] = tot[0][t] / tt;
      }
    }
  } else if constexpr (OP == F_HALF) {
    if (on && st_flag) {
      if (sqrt(tot[0][t]) < st_thr) {
        S.halfconv[t] = 1;
        S.any[4] = 1;
      } else if (st_pend) {
        S.skip[t] = 1;
        S.rst[t] = 1;
        S.any[2] = 1;
      }
    }
  } else if constexpr (OP == F_XR) {
    if (on && !st_flag) {
      const double rho_new = tot[0][t];
      S.rho_old[t] = st_rho;
      S.rho[t] = rho_new;
      S.beta[t] = (rho_new / st_rho) * (st_alpha / st_omega);
      if (sqrt(tot[1][t]) < st_thr) {
        S.full[t] = 1;
        S.any[1] = 1;  // breakdown checks follow the true-residual check
      } else if (fabs(st_omega) < TINY || fabs(rho_new) < TINY || forced) {
        S.rst[t] = 1;
        S.any[2] = 1;
      }
    }
  } else if constexpr (OP == F_FULL) {
    if (on && st_flag) {
      if (sqrt(tot[0][t]) < st_thr) {
        S.status[t] = ST_CONV;  // iteration count set at the end of the iteration
      } else {
        const double rho_new = tot[1][t];
        S.rho[t] = rho_new;
        S.beta[t] = (rho_new / st_rho_old) * (st_alpha / st_omega);
        if (fabs(st_omega) < TINY || fabs(rho_new) < TINY || forced) {
          S.rst[t] = 1;
          S.any[2] = 1;
        }
      }
    }
  } else if constexpr (OP == F_RESTART_END) {
    if (S.any[2] != 0 && st_flag && st_status == ST_ACTIVE) {
      const double rr = tot[0][t];
      S.rho[t] = rr;
      S.rho_old[t] = S.alpha[t] = S.omega[t] = 1.0;
      S.beta[t] = rr;
      S.restarts[t] = st_restarts + 1;
      if (st_restarts + 1 > 1) S.status[t] = ST_BREAK;
    }
  }
  if constexpr (OP == F_RESTART_END) iter_end_body(k, S, it, maxit);
}

__global__ void k_iter_end(int k, State S, int it, int maxit) { iter_end_body(k, S, it, maxit); }

}  // namespace
}  // namespace sai
