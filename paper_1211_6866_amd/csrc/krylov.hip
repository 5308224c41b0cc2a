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
// GMRES(m) has two forms: for small n one workgroup per column for the whole
// solve (modified Gram-Schmidt Arnoldi, Givens rotations, solution update at
// the end of each cycle, convergence on the true residual), and for large n the
// batched form of gmres_batched.hpp, whose sparse products are the BiCGStab
// ones.
#include "sai_internal.hpp"

#include "bicgstab_kernels.hpp"

namespace sai {
namespace {

// ---- batched BiCGStab driver ---------------------------------------------------------
//
// The k systems start in one n x kp block.  When enough columns have stopped that
// the remaining ones fit a narrower lane class, the block is narrowed: the stopped
// columns' x (and status, iteration count) are handed out, the active columns'
// vectors and scalars are gathered into a new block, and the iteration continues
// there with fewer lanes per row.  Each column's arithmetic is unchanged (its
// products, updates and stopping tests do not depend on the other columns; only
// the order of the partial sums of its dot products follows the grid).

// lanes per row for k columns: the smallest of 1, 2, 4, 6, 8, 12, 16, 32 covering
// the column pairs, and at least LP_MIN (knob, default 1: with 2 a one-column
// block takes tiles of 128 rows, whose entries of M fit the LDS staging area)
int lp_class(int k) {
  const int pairs = (k + 1) / 2;
  const int lmin = tune_get("LP_MIN", 1);
  const int cls[] = {1, 2, 4, 6, 8, 12, 16, 32};
  for (int c : cls)
    if (pairs <= c && c >= lmin) return c;
  return 32;
}

// For each of nv vector pairs: dst[i, to[q]] = src[i, from[q]] for q < np (and
// dst[i, zero_col] = 0 when zero_col >= 0); one thread per (row, column)
struct ColCopy {
  const double* src[10];
  double* dst[10];
};
__global__ void __launch_bounds__(NT) k_cols_copy(int64_t n, ColCopy cc, int nv, int lds, int ldd,
                                                  const int* __restrict__ from, const int* __restrict__ to,
                                                  int np, int zero_col) {
  const int w = np + (zero_col >= 0 ? 1 : 0);
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n * w; t += (int64_t)gridDim.x * NT) {
    const int64_t i = t / w;
    const int q = (int)(t % w);
    for (int v = 0; v < nv; ++v) {
      if (q < np) cc.dst[v][i * ldd + to[q]] = cc.src[v][i * lds + from[q]];
      else cc.dst[v][i * ldd + zero_col] = 0.0;
    }
  }
}

// One block of systems: n x kp vectors (b, x, r, r_hat, p, v, s, p_hat, s_hat, t),
// per-column scalars and flags, and the caller's column of each block column.
struct Block {
  int k = 0, kp = 0;
  std::vector<int> cols;
  DBuf<double> vec[10];
  DBuf<double> sc;  // rho, rho_old, alpha, omega, beta, thr (64 each)
  DBuf<int> si;     // status, iters, skip, restarts, half, full, rst, halfconv, wasact, pend (64 each), any
  State S{};
  Vec V{};
};
constexpr int SC_N = 6 * 64, SI_N = 10 * 64 + 8;

// Set B up for k columns; the vector buffers are (re)allocated only when their
// capacity (cap columns) is smaller than needed.
void block_alloc(Block& B, int k, int64_t n, const Allocator& al, double* part, hipStream_t st,
                 int& cap) {
  B.k = k;
  B.kp = k + (k & 1);
  if (cap < B.kp) {
    const size_t nk = (size_t)n * B.kp;
    for (auto& v : B.vec) v.alloc(&al, nk);
    cap = B.kp;
  }
  if (!B.sc.p) B.sc.alloc(&al, SC_N);
  if (!B.si.p) B.si.alloc(&al, SI_N);
  HIPC(hipMemsetAsync(B.sc.p, 0, sizeof(double) * SC_N, st));
  HIPC(hipMemsetAsync(B.si.p, 0, sizeof(int) * SI_N, st));
  State& S = B.S;
  S.rho = B.sc.p;
  S.rho_old = B.sc.p + 64;
  S.alpha = B.sc.p + 128;
  S.omega = B.sc.p + 192;
  S.beta = B.sc.p + 256;
  S.thr = B.sc.p + 320;
  S.status = B.si.p;
  S.iters = B.si.p + 64;
  S.skip = B.si.p + 128;
  S.restarts = B.si.p + 192;
  S.half = B.si.p + 256;
  S.full = B.si.p + 320;
  S.rst = B.si.p + 384;
  S.halfconv = B.si.p + 448;
  S.wasact = B.si.p + 512;
  S.pend = B.si.p + 576;
  S.any = B.si.p + 640;
  S.part = part;
  B.V = Vec{B.vec[0].p, B.vec[1].p, B.vec[2].p, B.vec[3].p, B.vec[4].p,
            B.vec[5].p, B.vec[6].p, B.vec[7].p, B.vec[8].p, B.vec[9].p};
}

enum { IT_DONE = 0, IT_NARROW = 1 };

// Profile names of one iteration's launches; the launches on a narrowed block
// and those of transposed solves (the adjoint: products with M^T and A~^T)
// carry their own names, so that the per-launch figures of the full-width
// forward block (whose algorithmic bytes follow from k) stay apart.
struct IterNames {
  const char *init, *pup, *m32, *m64, *av, *fin, *s, *at, *half, *xr, *full, *rst, *fend;
};
const IterNames kWideNames{"bicg_init", "bicg_p_update", "bicg_spmm_M_f32", "bicg_spmm_M_f64",
                           "bicg_spmm_A_dot1", "bicg_finish", "bicg_s_update", "bicg_spmm_A_dot2",
                           "bicg_halfcheck", "bicg_xr_update", "bicg_fullcheck", "bicg_restart",
                           "bicg_finish_end"};
const IterNames kNarrowNames{"bicg_narrow_init", "bicg_narrow_p_update", "bicg_spmm_narrow_M_f32",
                             "bicg_spmm_narrow_M_f64", "bicg_spmm_narrow_A_dot1", "bicg_narrow_finish",
                             "bicg_narrow_s_update", "bicg_spmm_narrow_A_dot2", "bicg_narrow_halfcheck",
                             "bicg_narrow_xr_update", "bicg_narrow_fullcheck", "bicg_narrow_restart",
                             "bicg_narrow_finish_end"};
const IterNames kWideNamesT{"bicg_t_init", "bicg_t_p_update", "bicg_t_spmm_M_f32", "bicg_t_spmm_M_f64",
                            "bicg_t_spmm_A_dot1", "bicg_t_finish", "bicg_t_s_update", "bicg_t_spmm_A_dot2",
                            "bicg_t_halfcheck", "bicg_t_xr_update", "bicg_t_fullcheck", "bicg_t_restart",
                            "bicg_t_finish_end"};
const IterNames kNarrowNamesT{"bicg_t_narrow_init", "bicg_t_narrow_p_update", "bicg_t_spmm_narrow_M_f32",
                              "bicg_t_spmm_narrow_M_f64", "bicg_t_spmm_narrow_A_dot1", "bicg_t_narrow_finish",
                              "bicg_t_narrow_s_update", "bicg_t_spmm_narrow_A_dot2",
                              "bicg_t_narrow_halfcheck", "bicg_t_narrow_xr_update", "bicg_t_narrow_fullcheck",
                              "bicg_t_narrow_restart", "bicg_t_narrow_finish_end"};

// Iterations it, it+1, ... on block B with LP lanes per row, until every column
// has stopped or maxit is reached (IT_DONE), or the active columns would fit a
// narrower lane class (IT_NARROW).  The first phase also initialises from R.
template <int LP, class TM>
int iterate(Block& B, const Csr<double>& A, const Csr<TM>& M, int64_t n, int& it, int maxit, bool first,
            bool narrow_ok, const IterNames& N, const double* R, hipStream_t st, int* slot, hipEvent_t* ev) {
  const int k = B.k, kp = B.kp;
  State S = B.S;
  // output blocks larger than the 8 XCDs' L2s together are stored non-temporally
  // (NT_STORE: -1 by size, 0 never, 1 always).  Streamed reads non-temporal
  // (NT_LOAD = 1, set per workload class by the tuning file): faster on the
  // 100^3 matrix (96 MB blocks), slower on the 160^3 one (1.7 GB), on the
  // irregular 200,000 matrix (35 MB) and on the 500^2 one (20 MB)
  {
    const int ntk = tune_get("NT_STORE", -1);
    S.nt = ntk >= 0 ? ntk : ((size_t)n * kp * sizeof(double) > (size_t(32) << 20) ? 1 : 0);
    S.ntl = tune_get("NT_LOAD", 0) != 0 ? 1 : 0;
  }
  const Vec V = B.V;
  constexpr int RPB = (64 / LP) * (NT / 64);
  // streaming kernels: a grid-stride loop over rows (fewer blocks also means
  // fewer partial sums for the finishers to add).  512 blocks: the vector
  // updates ran ~7% faster than with 1024 on the 100^3 and 160^3 matrices.
  const int grid = (int)std::min<int64_t>(tune_get("SGRID", 512), (n + RPB - 1) / RPB);
  // Sparse products work on tiles of RPB rows (one per lane).  Their grid is
  // persistent: no more workgroups than fit on the device at once, so that the
  // grid sweeps the rows in one pass; it is a multiple of the XCD count.  When
  // an n x kp block fits in the 256 MB last-level (MALL) cache, XCD-contiguous
  // tile ranges let each XCD sweep one contiguous eighth of the rows and keep
  // its band of gathered rows in its own L2; larger blocks are swept by all
  // XCDs together (interleaved tiles), so that one band, not eight, must stay
  // resident in the MALL.
  const bool persist = tune_get("PERSIST", 1) != 0;
  const size_t nk = (size_t)n * kp;
  // tile-to-XCD map (TILE_LOOP): contiguous chunks per XCD when a block fits the
  // MALL, else round-robin tiles (XCHUNK = 0), or the blocked interleave with
  // runs of XCHUNK rows per XCD (set per workload class by the tuning file).  On
  // the 160^3 workload (1.7 GB blocks) runs of 800-3200 rows take the M product
  // from 2.82 to 2.56 ms with gathers in batches of 2 (slower with 8/4).
  constexpr int RPB_ = (64 / LP) * (NT / 64);
  const int xchunk = tune_get("XCHUNK", 0);
  const int xmap_big = xchunk > 0 ? std::max(2, xchunk / RPB_) : 0;
  const int xmap = tune_get("XMAP", nk * sizeof(double) <= (size_t(256) << 20) ? 1 : xmap_big);
  auto sp_grid = [&](const void* kern) {
    const int64_t ntiles = (n + RPB - 1) / RPB;
    int64_t g = std::min<int64_t>(NBMAX, ntiles);
    if (persist) g = std::min<int64_t>(g, resident_blocks(kern, NT));
    return (int)(g >= 8 ? (g & ~int64_t(7)) : g);
  };
  // test hooks: treat iterations BRK_TEST and BRK_TEST2 as breakdowns of every
  // active column (the restart path, and a second breakdown); 0, the default,
  // never matches
  const int force_it = tune_get("BRK_TEST", 0);
  const int force_it2 = tune_get("BRK_TEST2", 0);
  // M product: gather batch sizes (CH while >= CH entries remain, then CH2).
  // Blocks over 32 columns (LP = 32) take their own knob: there fewer loads in
  // flight per wavefront are faster (52 columns at 160^3: batches of 2 take
  // 2.82 ms against 3.20 with 8/4; the gathers are bound by the misses the
  // vector L1 keeps in flight), while one-column blocks wait on each batch
  // (0.28 ms with 8/4, 1.18 ms with batches of 2).
  const int mvar = LP >= 32 ? tune_get("SPMM_M_WIDE", 4) : tune_get("SPMM_M", 1);
  // One-column blocks (kp = 2) take the M product on the two-lane geometry
  // (SPMM_M_LP2, 1 by default): tiles of 128 rows, whose entries of M fit the
  // staging area, with the lane of the pad pair idle; the other kernels keep
  // one lane per row.  The block layout is the same, and so are the sums.  On
  // the 160^3 matrix the adjoint's M^T product went 0.282 -> 0.257 ms (with
  // LP_MIN = 2, which moves the other kernels too, the adjoint was slower).
  const bool m_lp2 = LP == 1 && tune_get("SPMM_M_LP2", 1) != 0;
  auto spmm_m = [&](const double* Xin, double* Y) {
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(sp_grid((const void*)kern)), dim3(NT), 0, st, n, k, kp, M, Xin, Y,
                         S, xmap);
    };
    if constexpr (LP == 1) {
      if (m_lp2) {
        constexpr int RPB2 = (64 / 2) * (NT / 64);
        const int xmap2 = tune_get("XMAP", nk * sizeof(double) <= (size_t(256) << 20)
                                               ? 1
                                               : (xchunk > 0 ? std::max(2, xchunk / RPB2) : 0));
        auto go2 = [&](auto kern) {
          int64_t g = std::min<int64_t>(NBMAX, (n + RPB2 - 1) / RPB2);
          if (persist) g = std::min<int64_t>(g, resident_blocks((const void*)kern, NT));
          g = g >= 8 ? (g & ~int64_t(7)) : g;
          hipLaunchKernelGGL(kern, dim3((int)g), dim3(NT), 0, st, n, k, kp, M, Xin, Y, S, xmap2);
        };
        switch (mvar) {
          case 0: go2(k_spmm<2, TM, 8, 4>); break;
          case 2: go2(k_spmm<2, TM, 5, 0>); break;
          case 3: go2(k_spmm<2, TM, 16, 8>); break;
          case 4: go2(k_spmm<2, TM, 2, 0>); break;
          default: go2(k_spmm<2, TM, 6, 3>); break;
        }
        return;
      }
    }
    switch (mvar) {
      case 0: go(k_spmm<LP, TM, 8, 4>); break;
      case 2: go(k_spmm<LP, TM, 5, 0>); break;
      case 3: go(k_spmm<LP, TM, 16, 8>); break;
      case 4: go(k_spmm<LP, TM, 2, 0>); break;
      default: go(k_spmm<LP, TM, 6, 3>); break;
    }
  };
  // A~ products (with their dot products): gather batch sizes
  const int avar = LP >= 32 ? tune_get("SPMM_A_WIDE", 5) : tune_get("SPMM_A", 0);
  // (3 and 4: the 8/4 and 7/0 batches reading A~ from global memory, no LDS staging;
  // 5: batches of 2)
  const void* kav = avar == 1   ? (const void*)k_av<LP, 8, 4>
                    : avar == 2 ? (const void*)k_av<LP, 7, 0>
                    : avar == 3 ? (const void*)k_av<LP, 8, 4, false>
                    : avar == 4 ? (const void*)k_av<LP, 7, 0, false>
                    : avar == 5 ? (const void*)k_av<LP, 2, 0>
                                : (const void*)k_av<LP, 4, 2>;
  const void* kat = avar == 1   ? (const void*)k_at<LP, 8, 4>
                    : avar == 2 ? (const void*)k_at<LP, 7, 0>
                    : avar == 3 ? (const void*)k_at<LP, 8, 4, false>
                    : avar == 4 ? (const void*)k_at<LP, 7, 0, false>
                    : avar == 5 ? (const void*)k_at<LP, 2, 0>
                                : (const void*)k_at<LP, 4, 2>;
  const int tgrid = std::min(sp_grid(kav), sp_grid(kat));
  auto go_a = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
  };
  auto spmm_av = [&]() {
    switch (avar) {
      case 1: go_a(k_av<LP, 8, 4>); break;
      case 2: go_a(k_av<LP, 7, 0>); break;
      case 3: go_a(k_av<LP, 8, 4, false>); break;
      case 4: go_a(k_av<LP, 7, 0, false>); break;
      case 5: go_a(k_av<LP, 2, 0>); break;
      default: go_a(k_av<LP, 4, 2>); break;
    }
  };
  auto spmm_at = [&]() {
    switch (avar) {
      case 1: go_a(k_at<LP, 8, 4>); break;
      case 2: go_a(k_at<LP, 7, 0>); break;
      case 3: go_a(k_at<LP, 8, 4, false>); break;
      case 4: go_a(k_at<LP, 7, 0, false>); break;
      case 5: go_a(k_at<LP, 2, 0>); break;
      default: go_a(k_at<LP, 4, 2>); break;
    }
  };
  if (first) {
    {
      SAI_PROF(N.init, st);
      hipLaunchKernelGGL((k_init<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, R, V, S);
      hipLaunchKernelGGL((k_fin<1, F_INIT>), dim3(1), dim3(FNT), 0, st, k, S, grid, 0, 0);
    }
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, st, k, S, 0, maxit);
    LAUNCH_CHECK();
    HIPC(hipMemcpyAsync(slot, S.any + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (slot[0] == 0) return IT_DONE;
  }
  // The active-column count of iteration it is read back while iteration it+1
  // runs (two pinned slots, one event each), so the device never waits for the
  // host.  An iteration queued after the last column stopped finds no active
  // column and does no work.
  const int it0 = it;
  for (; it <= maxit; ++it) {
#define LK(name, ...)              \
  do {                             \
    SAI_PROF(name, st);            \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)
    constexpr bool MF = sizeof(TM) == 4;
    LK(N.pup, (k_pupdate<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    {
      SAI_PROF(MF ? N.m32 : N.m64, st);
      spmm_m(V.p, V.ph);
    }
    {
      SAI_PROF(N.av, st);
      spmm_av();
    }
    LK(N.fin, (k_fin<1, F_AV>), dim3(1), dim3(FNT), 0, st, k, S, tgrid, 0, 0);
    LK(N.s, (k_s<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    {
      SAI_PROF(MF ? N.m32 : N.m64, st);
      spmm_m(V.s, V.sh);
    }
    {
      SAI_PROF(N.at, st);
      spmm_at();
    }
    LK(N.fin, (k_fin<3, F_AT>), dim3(1), dim3(FNT), 0, st, k, S, tgrid, 0, 0);
    LK(N.half, (k_halfcheck<LP>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
    LK(N.fin, (k_fin<1, F_HALF>), dim3(1), dim3(FNT), 0, st, k, S, tgrid, 0, 0);
    LK(N.xr, (k_xr<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    LK(N.fin, (k_fin<2, F_XR>), dim3(1), dim3(FNT), 0, st, k, S, grid, it, 0, force_it, force_it2);
    LK(N.full, (k_fullcheck<LP>), dim3(tgrid), dim3(NT), 0, st, n, k, kp, A, V, S, xmap);
    LK(N.fin, (k_fin<2, F_FULL>), dim3(1), dim3(FNT), 0, st, k, S, tgrid, it, 0, force_it,
       force_it2);
    LK(N.rst, (k_restart<LP>), dim3(grid), dim3(NT), 0, st, n, k, kp, V, S);
    LK(N.fend, (k_fin<1, F_RESTART_END>), dim3(1), dim3(FNT), 0, st, k, S, grid, it, maxit);
#undef LK
    LAUNCH_CHECK();
    HIPC(hipMemcpyAsync(slot + (it & 1), S.any + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipEventRecord(ev[it & 1], st));
    if (it > it0) {
      // count after iteration it-1 (iteration it is already queued behind it)
      HIPC(hipEventSynchronize(ev[(it - 1) & 1]));
      const int act = slot[(it - 1) & 1];
      if (act == 0) {
        ++it;
        return IT_DONE;
      }
      // narrow when the active columns fit a smaller lane class and the rows x
      // columns dropped from every later iteration repay the cost of moving the
      // block (about one iteration of idle device plus a copy).  Threshold: on
      // the irregular 200,000 matrix the last narrowing to one column pair
      // (1.2M dropped) saves 6.6 ms of a 97.6 ms step; any narrowing of the
      // 10^6-row matrices drops at least 2M.
      const int64_t drop = n * (int64_t)(kp - (act + (act & 1)));
      if (narrow_ok && LP > 1 && lp_class(act) < LP && 2 * act <= k &&
          drop >= (int64_t)tune_get("NARROW_MIN", 1000000)) {
        ++it;
        return IT_NARROW;
      }
    }
  }
  return IT_DONE;
}

template <class TM>
int iterate_lp(int lp, Block& B, const Csr<double>& A, const Csr<TM>& M, int64_t n, int& it, int maxit,
               bool first, bool narrow_ok, const IterNames& N, const double* R, hipStream_t st, int* slot,
               hipEvent_t* ev) {
  switch (lp) {
    case 1: return iterate<1, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    case 2: return iterate<2, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    case 4: return iterate<4, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    case 6: return iterate<6, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    case 8: return iterate<8, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    case 12: return iterate<12, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    case 16: return iterate<16, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
    default: return iterate<32, TM>(B, A, M, n, it, maxit, first, narrow_ok, N, R, st, slot, ev);
  }
}

// copy columns from[q] of each source (row stride lds) to columns to[q] of the
// matching destination (row stride ldd); idx: a device array of 128 ints, hidx
// a pinned host array of 128 ints that must stay unchanged until the copy ran
void cols_copy(int64_t n, const ColCopy& cc, int nv, int lds, int ldd, const std::vector<int>& from,
               const std::vector<int>& to, int zero_col, int* idx, int* hidx, hipStream_t st) {
  const int np = (int)from.size();
  if (np == 0 && zero_col < 0) return;
  for (int q = 0; q < np; ++q) {
    hidx[q] = from[q];
    hidx[64 + q] = to[q];
  }
  HIPC(hipMemcpyAsync(idx, hidx, sizeof(int) * 2 * 64, hipMemcpyHostToDevice, st));
  const int64_t work = n * (np + (zero_col >= 0 ? 1 : 0));
  hipLaunchKernelGGL(k_cols_copy, dim3(grid_for(work, NT, 8192)), dim3(NT), 0, st, n, cc, nv, lds, ldd,
                     idx, idx + 64, np, zero_col);
  LAUNCH_CHECK();
}

template <class TM>
int bicgstab(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R, double* X,
             const double* thr, int maxit, const Allocator& al, hipStream_t st, int* iters, int* status,
             bool transposed) {
  DBuf<double> part(&al, (size_t)3 * NBMAX * PSTRIDE);
  // two sets of block buffers, used alternately when the block narrows
  Block blk[2];
  int cap[2] = {0, 0};
  int cur = 0;
  block_alloc(blk[0], k, n, al, part.p, st, cap[0]);
  blk[0].cols.resize(k);
  for (int c = 0; c < k; ++c) blk[0].cols[c] = c;
  HIPC(hipMemcpyAsync(blk[0].S.thr, thr, sizeof(double) * k, hipMemcpyHostToDevice, st));
  DBuf<int> idx(&al, 2 * 2 * 64);
  HostStage hs(16 + 2 * 2 * 64 * sizeof(int) + sizeof(double) * SC_N + sizeof(int) * SI_N);
  int* slot = hs.as<int>();
  int* hidx = slot + 4;                                   // 2 x 128 ints
  double* hsc = reinterpret_cast<double*>(hidx + 256);    // SC_N
  int* hsi = reinterpret_cast<int*>(hsc + SC_N);           // SI_N
  hipEvent_t ev[2];
  HIPC(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIPC(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } evg{ev};
  const bool narrow_ok = tune_get("NARROW", 1) != 0;
  std::vector<int> rstat(k, ST_MAXIT), riter(k, 0);
  int it = 1;
  bool first = true, first_block = true;
  for (;;) {
    Block& B = blk[cur];
    const IterNames& nm = transposed ? (first_block ? kWideNamesT : kNarrowNamesT)
                                     : (first_block ? kWideNames : kNarrowNames);
    const int r = iterate_lp<TM>(lp_class(B.k), B, A, M, n, it, maxit, first, narrow_ok, nm, R, st,
                                 slot, ev);
    first_block = false;
    first = false;
    HIPC(hipMemcpyAsync(hsc, B.sc.p, sizeof(double) * SC_N, hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(hsi, B.si.p, sizeof(int) * SI_N, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    // hand out the stopped columns (all of them at the end)
    std::vector<int> keep, from, to;
    for (int c = 0; c < B.k; ++c) {
      if (r == IT_NARROW && hsi[c] == ST_ACTIVE) {
        keep.push_back(c);
      } else {
        rstat[B.cols[c]] = hsi[c];
        riter[B.cols[c]] = hsi[64 + c];
        from.push_back(c);
        to.push_back(B.cols[c]);
      }
    }
    {
      ColCopy cc{};
      cc.src[0] = B.V.x;
      cc.dst[0] = X;
      cols_copy(n, cc, 1, B.kp, k, from, to, -1, idx.p, hidx, st);
    }
    if (keep.empty()) break;
    // narrow: gather the active columns' vectors and scalars into the other set
    Block& NB = blk[1 - cur];
    block_alloc(NB, (int)keep.size(), n, al, part.p, st, cap[1 - cur]);
    NB.cols.resize(keep.size());
    std::vector<int> to2(keep.size());
    for (size_t q = 0; q < keep.size(); ++q) {
      NB.cols[q] = B.cols[keep[q]];
      to2[q] = (int)q;
    }
    const int zc = (NB.k & 1) ? NB.k : -1;  // the pad column of the new block
    {
      ColCopy cc{};
      for (int v = 0; v < 10; ++v) {
        cc.src[v] = B.vec[v].p;
        cc.dst[v] = NB.vec[v].p;
      }
      cols_copy(n, cc, 10, B.kp, NB.kp, keep, to2, zc, idx.p + 128, hidx + 128, st);
    }
    // scalars of the kept columns, in the pinned stage (read back above)
    std::vector<double> nsc(SC_N, 0.0);
    std::vector<int> nsi(SI_N, 0);
    for (size_t q = 0; q < keep.size(); ++q) {
      for (int a = 0; a < 6; ++a) nsc[a * 64 + q] = hsc[a * 64 + keep[q]];
      for (int a = 0; a < 10; ++a) nsi[a * 64 + q] = hsi[a * 64 + keep[q]];
    }
    nsi[640 + 3] = (int)keep.size();  // active count; the flags are clear between iterations
    std::memcpy(hsc, nsc.data(), sizeof(double) * SC_N);
    std::memcpy(hsi, nsi.data(), sizeof(int) * SI_N);
    HIPC(hipMemcpyAsync(NB.sc.p, hsc, sizeof(double) * SC_N, hipMemcpyHostToDevice, st));
    HIPC(hipMemcpyAsync(NB.si.p, hsi, sizeof(int) * SI_N, hipMemcpyHostToDevice, st));
    cur = 1 - cur;
  }
  HIPC(hipStreamSynchronize(st));
  int worst = SAI_OK;
  for (int c = 0; c < k; ++c) {
    const int code = rstat[c] == ST_CONV ? 0 : (rstat[c] == ST_BREAK ? 2 : 1);
    if (status) status[c] = code;
    if (iters) iters[c] = riter[c];
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
              int* iters, int* status, bool transposed) {
  if (restart < 1 || restart > GM_MAXM) SAI_THROW(SAI_EINVAL, "GMRES restart must be in [1, %d]", GM_MAXM);
  DBuf<double> work(&al, (size_t)k * (restart + 3) * n);
  DBuf<double> dthr(&al, k);
  DBuf<int> dit(&al, k), dst(&al, k);
  HIPC(hipMemcpyAsync(dthr.p, thr, sizeof(double) * k, hipMemcpyHostToDevice, st));
  SAI_PROF(transposed ? "gmres_t_fused" : "gmres_fused", st);
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

}  // namespace
}  // namespace sai

#include "gmres_batched.hpp"

namespace sai {
namespace {

// GMRES(m): the batched form once n k reaches GMRES_BATCH_NK (default 32768),
// the per-column workgroups below it.  Measured with GMRES(30): per-column was
// faster for 2,025 and 4,900 rows with 4 columns (3.4 vs 7.8 ms, 10.5 vs 13.0 ms),
// batched for 10,000 rows with 4 columns (11.5 vs 14.4 ms) and 3,375 rows with
// 11 columns (2.4 vs 3.3 ms), and 13x faster at 216,000 rows with 11 columns.
template <class TM>
int gmres_solve(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R, double* X,
                const double* thr, int restart, int maxit, const Allocator& al, hipStream_t st, int* iters,
                int* status, bool transposed) {
  if (restart < 1 || restart > GM_MAXM) SAI_THROW(SAI_EINVAL, "GMRES restart must be in [1, %d]", GM_MAXM);
  if (n * k >= (int64_t)tune_get("GMRES_BATCH_NK", 32768))
    return gmres_batched<TM>(A, M, n, k, R, X, thr, restart, maxit, al, st, iters, status, transposed);
  return gmres_run<TM>(A, M, n, k, R, X, thr, restart, maxit, al, st, iters, status, transposed);
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
    return gmres_solve<TM>(A, M, n, k, R, X, thr, o.restart, o.maxit, al, st, iters, status, transpose != 0);
  return bicgstab<TM>(A, M, n, k, R, X, thr, o.maxit, al, st, iters, status, transpose != 0);
}

// dst (n x kc, row stride kc) = columns c0 .. c0+kc-1 of src (row stride lds),
// or back (to_src): those columns of src = dst
__global__ void k_col_group(int64_t n, int lds, int c0, int kc, const double* __restrict__ a,
                            double* __restrict__ b, int to_src) {
  const int64_t nk = n * kc;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < nk; t += (int64_t)gridDim.x * NT) {
    const int64_t i = t / kc, e = i * lds + c0 + t % kc;
    if (to_src) b[e] = a[t];
    else b[t] = a[e];
  }
}

int krylov_one(const sai_split_s* sp, const sai_precond_s* pc, int transpose, int k, const double* R,
               double* X, const double* thr, const sai_solve_opts& o, hipStream_t st, int32_t* iters,
               int32_t* status) {
  if (pc->precision == SAI_FP32)
    return krylov_typed<float>(sp, pc, transpose, k, R, X, thr, o, st, iters, status);
  return krylov_typed<double>(sp, pc, transpose, k, R, X, thr, o, st, iters, status);
}

}  // namespace

// Blocks of up to KMAX columns run as one lockstep solve; wider blocks in groups
// of KMAX columns, one after the other (the systems are independent, so each
// column's iterates do not depend on the grouping).
constexpr int KMAX = 64;

int krylov_impl(const sai_split_s* sp, const sai_precond_s* pc, int transpose, int k,
                const double* R, double* X, const double* thr, const sai_solve_opts& o,
                hipStream_t st, int32_t* iters, int32_t* status) {
  if (k < 1) SAI_THROW(SAI_EINVAL, "k must be >= 1 (got %d)", k);
  if (o.method != SAI_BICGSTAB && o.method != SAI_GMRES) SAI_THROW(SAI_EINVAL, "bad method");
  if (o.maxit < 0) SAI_THROW(SAI_EINVAL, "maxit < 0");
  if (pc->n != sp->n) SAI_THROW(SAI_EINVAL, "preconditioner and split sizes differ");
  if (k <= KMAX) return krylov_one(sp, pc, transpose, k, R, X, thr, o, st, iters, status);
  const Allocator al{sp->al.a, st};
  const int64_t n = sp->n;
  DBuf<double> Rg(&al, (size_t)n * KMAX), Xg(&al, (size_t)n * KMAX);
  int worst = SAI_OK;
  for (int c0 = 0; c0 < k; c0 += KMAX) {
    const int kc = std::min(KMAX, k - c0);
    const unsigned g = grid_for(n * kc, NT, 8192);
    hipLaunchKernelGGL(k_col_group, dim3(g), dim3(NT), 0, st, n, k, c0, kc, R, Rg.p, 0);
    LAUNCH_CHECK();
    const int code = krylov_one(sp, pc, transpose, kc, Rg.p, Xg.p, thr + c0, o, st,
                                iters ? iters + c0 : nullptr, status ? status + c0 : nullptr);
    hipLaunchKernelGGL(k_col_group, dim3(g), dim3(NT), 0, st, n, k, c0, kc, (const double*)Xg.p, X, 1);
    LAUNCH_CHECK();
    if (code == SAI_EBREAKDOWN || (code == SAI_ENOCONV && worst == SAI_OK)) worst = code;
  }
  HIPC(hipStreamSynchronize(st));
  return worst;
}

}  // namespace sai
