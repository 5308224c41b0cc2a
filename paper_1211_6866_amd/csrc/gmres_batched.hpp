// Batched right-preconditioned GMRES(m) for the k columns of a block (included by
// krylov.hip after the BiCGStab driver).  Section 5 names GMRES(20) among the
// solvers tried on the s+1 systems; this form runs the k systems in lockstep, so
// that each product with M and with A~ streams the matrix once for all columns
// (the same tiled products as BiCGStab), where the per-column form runs one
// workgroup per column through the whole solve.
//
// The systems live in n x kp row-major blocks (kp = k rounded up to even; the
// pad column is never active).  Per Arnoldi step j of a cycle, for the columns
// still in the cycle:
//   Z = M V_j;  W = A~ Z;
//   h = V_{0..j}^T W;  W -= V h;  h' = V_{0..j}^T W;  W -= V h'   (classical
//   Gram-Schmidt with one reorthogonalisation: the projection of modified
//   Gram-Schmidt in exact arithmetic, as stable in practice, and two passes
//   over the basis instead of j + 1);
//   H[0..j, j] = h + h';  H[j+1, j] = ||W||;  Givens rotations as in the
//   per-column form;  V_{j+1} = W / H[j+1, j].
// A column leaves the cycle when its rotated residual estimate |g[j+1]| is
// below its threshold, H[j+1, j] = 0, maxit is reached or j + 1 = m.  At the
// end of the cycle every column of the cycle solves its triangular system,
// takes x += M (V y), and its true residual R - A~ x decides convergence (and
// restarts the next cycle from it).  Dot products are reduced per workgroup
// and the partial sums added in a fixed order (deterministic results); the
// small per-column work (rotations, triangular solves, status) runs in
// one-block kernels, one thread per column, so the host only reads the active
// count once per cycle.
#pragma once

namespace sai {
namespace {

constexpr int GB_NT = 256;
constexpr int GB_NB = 1024;    // most workgroups of a reduction (partial sums per column)
constexpr int GB_CH = 32;      // basis vectors per projection launch
constexpr int GB_Q = GM_MAXM + 1;

// per-column state, 64 entries each
struct GbState {
  int* arn;       // 0 while the column is in the Arnoldi steps of the cycle
  int* cyc;       // 0 for the columns of the current cycle
  int* zero;      // 64 zeros (no column skipped)
  int* any_arn;   // [3]: columns in the Arnoldi steps
  int* any_cyc;   // [3]: columns of the cycle
  int* st;        // ST_ACTIVE / ST_CONV / ST_MAXIT
  int* kk;        // steps of the current cycle
  int* it;        // iterations so far
  int* any_st;    // [3]: active columns
  double *thr, *beta, *a, *g, *cs, *sn, *y, *H, *hh, *hh2, *nn;
};

// B = R (pad column 0), X = 0, W = B
__global__ void __launch_bounds__(GB_NT) k_gb_load(int64_t n, int k, int kp, const double* __restrict__ R,
                                                  double* __restrict__ B, double* __restrict__ X,
                                                  double* __restrict__ W) {
  const int64_t nk = n * kp;
  for (int64_t t = (int64_t)blockIdx.x * GB_NT + threadIdx.x; t < nk; t += (int64_t)gridDim.x * GB_NT) {
    const int64_t i = t / kp;
    const int c = (int)(t % kp);
    const double b = c < k ? R[i * k + c] : 0.0;
    B[t] = b;
    X[t] = 0.0;
    W[t] = b;
  }
}

// ---- reductions over the rows ------------------------------------------------------
//
// The basis V_0, V_1, ... is one array, V_q at Vb + q nk (nk = n kp).  A
// reduction block has GB_RT threads; thread t owns column c = t % kp of the
// rows g, g + RG, ... of the block's slice (g = t / kp, RG = GB_RT / kp row
// groups), a wavefront's loads covering consecutive elements.  The number of
// basis vectors NV is a template parameter so that the NV + 1 loads of a row
// are issued together.  Per-column block sums go to part[blk][q][c] (column
// partials of row groups added in a fixed order), and k_gb_fin adds the blocks'
// partials in a fixed order.

constexpr int GB_RT = 512;

// block sum of v over the row groups of column c, written to part[blk][q][c]
__device__ __forceinline__ void gb_block_sum(double v, bool on, int kp, int rg, int q, double* red,
                                             double* __restrict__ part) {
  const int t = threadIdx.x;
  red[t] = on ? v : 0.0;
  __syncthreads();
  if (t < kp) {
    double s = 0.0;
    for (int r = 0; r < rg; ++r) s += red[r * kp + t];
    part[((int64_t)blockIdx.x * GB_Q + q) * 64 + t] = s;
  }
  __syncthreads();
}

#define GB_RED_SETUP                                        \
  __shared__ double red[GB_RT];                             \
  const int rg = GB_RT / kp;                                \
  const int c = (int)threadIdx.x % kp, ro = (int)threadIdx.x / kp; \
  const bool on = ro < rg && act[c] == 0;                   \
  const int64_t nk = n * kp;                                \
  (void)nk;

#define GB_ROWS for (int64_t i = (int64_t)blockIdx.x * rg + ro; i < n; i += (int64_t)gridDim.x * rg)

// part[blk][q0 + q][c] = V_{q0+q}[rows of blk, c]^T W[rows of blk, c], q < NV
template <int NV>
__global__ void __launch_bounds__(GB_RT) k_gb_dots(int64_t n, int kp, int q0, const double* __restrict__ Vb,
                                                  const double* __restrict__ W, const int* __restrict__ act,
                                                  const int* __restrict__ cnt, double* __restrict__ part) {
  if (cnt[3] == 0) return;
  GB_RED_SETUP
  const double* V0 = Vb + nk * q0;
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  if (on) {
    GB_ROWS {
      const int64_t e = i * kp + c;
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = V0[nk * q + e];
      const double w = W[e];
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] += v[q] * w;
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) gb_block_sum(acc[q], on, kp, rg, q0 + q, red, part);
}

// W -= V_{0..NV-1} h, then part[blk][q][c] = V_q^T W (the second Gram-Schmidt
// pass's products, on the projected W, from the same loads of V)
template <int NV>
__global__ void __launch_bounds__(GB_RT) k_gb_projdots(int64_t n, int kp, const double* __restrict__ Vb,
                                                      const double* __restrict__ h, double* __restrict__ W,
                                                      const int* __restrict__ act, const int* __restrict__ cnt,
                                                      double* __restrict__ part) {
  if (cnt[3] == 0) return;
  GB_RED_SETUP
  double hq[NV], acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    hq[q] = on ? h[q * 64 + c] : 0.0;
    acc[q] = 0.0;
  }
  if (on) {
    GB_ROWS {
      const int64_t e = i * kp + c;
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = Vb[nk * q + e];
      double w = W[e];
#pragma unroll
      for (int q = 0; q < NV; ++q) w -= hq[q] * v[q];
      W[e] = w;
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] += v[q] * w;
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) gb_block_sum(acc[q], on, kp, rg, q, red, part);
}

// W -= V_{q0..q0+NV-1} h[q0..]; with norm, part[blk][0][c] = sum of the new W^2
template <int NV>
__global__ void __launch_bounds__(GB_RT) k_gb_project(int64_t n, int kp, int q0, const double* __restrict__ Vb,
                                                     const double* __restrict__ h, double* __restrict__ W,
                                                     const int* __restrict__ act, const int* __restrict__ cnt,
                                                     int norm, double* __restrict__ part) {
  if (cnt[3] == 0) return;
  GB_RED_SETUP
  const double* V0 = Vb + nk * q0;
  double hq[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) hq[q] = on ? h[(q0 + q) * 64 + c] : 0.0;
  double acc = 0.0;
  if (on) {
    GB_ROWS {
      const int64_t e = i * kp + c;
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = V0[nk * q + e];
      double w = W[e];
#pragma unroll
      for (int q = 0; q < NV; ++q) w -= hq[q] * v[q];
      W[e] = w;
      acc += w * w;
    }
  }
  if (norm) gb_block_sum(acc, on, kp, rg, 0, red, part);
}

// W = B - AX and part[blk][0][c] = sum of W^2
__global__ void __launch_bounds__(GB_RT) k_gb_resid(int64_t n, int kp, const double* __restrict__ B,
                                                   const double* __restrict__ AX, double* __restrict__ W,
                                                   const int* __restrict__ act, const int* __restrict__ cnt,
                                                   double* __restrict__ part) {
  if (cnt[3] == 0) return;
  GB_RED_SETUP
  double acc = 0.0;
  if (on) {
    GB_ROWS {
      const int64_t e = i * kp + c;
      const double w = B[e] - AX[e];
      W[e] = w;
      acc += w * w;
    }
  }
  gb_block_sum(acc, on, kp, rg, 0, red, part);
}

#undef GB_ROWS
#undef GB_RED_SETUP

// out[q][c] = sum over the nb blocks of part[blk][q][c] (one block per q):
// thread (g, c) adds blocks g, g + G, ... in order (G = GB_RT / kp), then the
// G sums are added in order
__global__ void __launch_bounds__(GB_RT) k_gb_fin(int nb, int kp, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  __shared__ double red[GB_RT];
  const int q = blockIdx.x;
  const int G = GB_RT / kp;
  const int c = (int)threadIdx.x % kp, g = (int)threadIdx.x / kp;
  double s = 0.0;
  if (g < G)
    for (int b = g; b < nb; b += G) s += part[((int64_t)b * GB_Q + q) * 64 + c];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 64) {
    double r = 0.0;
    if ((int)threadIdx.x < kp)
      for (int u = 0; u < G; ++u) r += red[u * kp + threadIdx.x];
    out[q * 64 + threadIdx.x] = r;
  }
}

// dst = a[c] src for the columns with act[c] == 0
__global__ void __launch_bounds__(GB_NT) k_gb_scale(int64_t n, int kp, const double* __restrict__ a,
                                                   const double* __restrict__ src, double* __restrict__ dst,
                                                   const int* __restrict__ act, const int* __restrict__ cnt) {
  if (cnt[3] == 0) return;
  const int64_t nk = n * kp;
  for (int64_t t = (int64_t)blockIdx.x * GB_NT + threadIdx.x; t < nk; t += (int64_t)gridDim.x * GB_NT) {
    const int c = (int)(t % kp);
    if (act[c] == 0) dst[t] = a[c] * src[t];
  }
}

// Z[i, c] = sum_{q < kk[c]} y[q][c] V_q[i, c] for the columns with act[c] == 0
__global__ void __launch_bounds__(GB_NT) k_gb_combine(int64_t n, int kp, const double* __restrict__ Vb,
                                                     const double* __restrict__ y,
                                                     const int* __restrict__ kk, double* __restrict__ Z,
                                                     const int* __restrict__ act, const int* __restrict__ cnt) {
  if (cnt[3] == 0) return;
  const int64_t nk = n * kp;
  for (int64_t t = (int64_t)blockIdx.x * GB_NT + threadIdx.x; t < nk; t += (int64_t)gridDim.x * GB_NT) {
    const int c = (int)(t % kp);
    if (act[c] != 0) continue;
    const int kq = kk[c];
    double s = 0.0;
    int q = 0;
    for (; q + 4 <= kq; q += 4) {  // four independent loads at a time
      const double v0 = Vb[nk * q + t], v1 = Vb[nk * (q + 1) + t];
      const double v2 = Vb[nk * (q + 2) + t], v3 = Vb[nk * (q + 3) + t];
      s += y[q * 64 + c] * v0;
      s += y[(q + 1) * 64 + c] * v1;
      s += y[(q + 2) * 64 + c] * v2;
      s += y[(q + 3) * 64 + c] * v3;
    }
    for (; q < kq; ++q) s += y[q * 64 + c] * Vb[nk * q + t];
    Z[t] = s;
  }
}

// X += D for the columns with act[c] == 0
__global__ void __launch_bounds__(GB_NT) k_gb_add(int64_t n, int kp, const double* __restrict__ D,
                                                 double* __restrict__ X, const int* __restrict__ act,
                                                 const int* __restrict__ cnt) {
  if (cnt[3] == 0) return;
  const int64_t nk = n * kp;
  for (int64_t t = (int64_t)blockIdx.x * GB_NT + threadIdx.x; t < nk; t += (int64_t)gridDim.x * GB_NT)
    if (act[t % kp] == 0) X[t] += D[t];
}

// caller's X (n x k) from the block (n x kp)
__global__ void __launch_bounds__(GB_NT) k_gb_out(int64_t n, int k, int kp, const double* __restrict__ Xb,
                                                 double* __restrict__ X) {
  const int64_t nk = n * k;
  for (int64_t t = (int64_t)blockIdx.x * GB_NT + threadIdx.x; t < nk; t += (int64_t)gridDim.x * GB_NT)
    X[t] = Xb[(t / k) * kp + t % k];
}

// ---- one-block kernels, thread c for column c ---------------------------------------

__device__ __forceinline__ void gb_count(const int* flag, int k, int* any) {
  __shared__ int s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  if (threadIdx.x < k && flag[threadIdx.x] == 0) atomicAdd(&s, 1);
  __syncthreads();
  if (threadIdx.x == 0) any[3] = s;
}

// status from the initial residual norm (x = 0, r = R)
__global__ void __launch_bounds__(64) k_gb_setup(int k, int maxit, GbState G) {
  const int c = threadIdx.x;
  if (c < k) {
    const double b = sqrt(G.nn[c]);
    G.beta[c] = b;
    G.it[c] = 0;
    G.st[c] = b < G.thr[c] ? ST_CONV : (maxit <= 0 ? ST_MAXIT : ST_ACTIVE);
  }
  __syncthreads();
  gb_count(G.st, k, G.any_st);
}

// start a cycle for every active column: V_0 = r / beta (a = 1 / beta), g = beta e_1
__global__ void __launch_bounds__(64) k_gb_cycle_start(int k, int m, GbState G) {
  const int c = threadIdx.x;
  const bool on = c < k && G.st[c] == ST_ACTIVE;
  G.arn[c] = on ? 0 : 1;
  G.cyc[c] = on ? 0 : 1;
  G.kk[c] = 0;
  G.a[c] = on ? 1.0 / G.beta[c] : 0.0;
  for (int q = 0; q <= m; ++q) G.g[q * 64 + c] = q == 0 && on ? G.beta[c] : 0.0;
  __syncthreads();
  gb_count(G.arn, k, G.any_arn);
  gb_count(G.cyc, k, G.any_cyc);
}

// Arnoldi step j: the new column of H from the two projections and ||W||, the
// previous rotations, a new rotation, the residual estimate and the exit test
__global__ void __launch_bounds__(64) k_gb_step(int k, int m, int j, int maxit, GbState G) {
  const int c = threadIdx.x;
  if (c < k && G.arn[c] == 0) {
    double* H = G.H;
    auto h = [&](int q, int jj) -> double& { return H[((int64_t)q * GM_MAXM + jj) * 64 + c]; };
    for (int q = 0; q <= j; ++q) h(q, j) = G.hh[q * 64 + c] + G.hh2[q * 64 + c];
    const double hnext = sqrt(G.nn[c]);
    h(j + 1, j) = hnext;
    for (int q = 0; q < j; ++q) {
      const double a = h(q, j), b = h(q + 1, j);
      const double cq = G.cs[q * 64 + c], sq = G.sn[q * 64 + c];
      h(q, j) = cq * a + sq * b;
      h(q + 1, j) = -sq * a + cq * b;
    }
    const double a = h(j, j), b = h(j + 1, j);
    double cc = 1.0, ss = 0.0;
    if (b != 0.0) {
      const double r = hypot(a, b);
      cc = a / r;
      ss = b / r;
    }
    G.cs[j * 64 + c] = cc;
    G.sn[j * 64 + c] = ss;
    h(j, j) = cc * a + ss * b;
    h(j + 1, j) = 0.0;
    const double gj = G.g[j * 64 + c];
    G.g[(j + 1) * 64 + c] = -ss * gj;
    G.g[j * 64 + c] = cc * gj;
    G.kk[c] = j + 1;
    const int it = ++G.it[c];
    const bool leave = hnext == 0.0 || fabs(G.g[(j + 1) * 64 + c]) < G.thr[c] || it >= maxit || j + 1 == m;
    if (leave) G.arn[c] = 1;
    else G.a[c] = 1.0 / hnext;
  }
  __syncthreads();
  gb_count(G.arn, k, G.any_arn);
}

// y = H(0:kk, 0:kk)^{-1} g(0:kk) for the columns of the cycle
__global__ void __launch_bounds__(64) k_gb_backsolve(int k, GbState G) {
  const int c = threadIdx.x;
  if (c >= k || G.cyc[c] != 0) return;
  const int kk = G.kk[c];
  for (int q = kk - 1; q >= 0; --q) {
    double s = G.g[q * 64 + c];
    for (int u = q + 1; u < kk; ++u) s -= G.H[((int64_t)q * GM_MAXM + u) * 64 + c] * G.y[u * 64 + c];
    G.y[q * 64 + c] = s / G.H[((int64_t)q * GM_MAXM + q) * 64 + c];
  }
}

// convergence on the true residual at the end of a cycle
__global__ void __launch_bounds__(64) k_gb_cycle_end(int k, int maxit, GbState G) {
  const int c = threadIdx.x;
  if (c < k && G.cyc[c] == 0) {
    const double b = sqrt(G.nn[c]);
    G.beta[c] = b;
    G.st[c] = b < G.thr[c] ? ST_CONV : (G.it[c] >= maxit ? ST_MAXIT : ST_ACTIVE);
  }
  __syncthreads();
  gb_count(G.st, k, G.any_st);
}

// profile names: the forward's, and those of transposed solves (the adjoint)
struct GmresNames {
  const char *init, *start, *m32, *m64, *a, *orth, *step, *end;
};
const GmresNames kGmresNames{"gmres_init", "gmres_cycle_start", "gmres_spmm_M_f32", "gmres_spmm_M_f64",
                             "gmres_spmm_A", "gmres_orth", "gmres_step", "gmres_cycle_end"};
const GmresNames kGmresNamesT{"gmres_t_init", "gmres_t_cycle_start", "gmres_t_spmm_M_f32",
                              "gmres_t_spmm_M_f64", "gmres_t_spmm_A", "gmres_t_orth", "gmres_t_step",
                              "gmres_t_cycle_end"};

template <int LP, class TM>
int gmres_batched_lp(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R, double* X,
                     const double* thr, int m, int maxit, const Allocator& al, hipStream_t st, int* iters,
                     int* status, bool transposed) {
  const GmresNames& GN = transposed ? kGmresNamesT : kGmresNames;
  const int kp = k + (k & 1);
  const size_t nk = (size_t)n * kp;
  DBuf<double> basis(&al, nk * (size_t)(m + 1));
  DBuf<double> Bv(&al, nk), Xv(&al, nk), Wv(&al, nk), Zv(&al, nk);
  DBuf<double> part(&al, (size_t)GB_NB * GB_Q * 64);
  // thr, beta, a, nn; g; cs, sn, y; hh, hh2; H
  DBuf<double> sd(&al, (size_t)64 * (4 + GB_Q + 2 * GM_MAXM + GM_MAXM + 2 * GB_Q) +
                           (size_t)GB_Q * GM_MAXM * 64);
  DBuf<int> si(&al, 64 * 6 + 3 * 8);
  GbState G{};
  G.arn = si.p;
  G.cyc = si.p + 64;
  G.zero = si.p + 128;
  G.st = si.p + 192;
  G.kk = si.p + 256;
  G.it = si.p + 320;
  G.any_arn = si.p + 384;
  G.any_cyc = si.p + 392;
  G.any_st = si.p + 400;
  double* d = sd.p;
  G.thr = d; d += 64;
  G.beta = d; d += 64;
  G.a = d; d += 64;
  G.nn = d; d += 64;
  G.g = d; d += 64 * GB_Q;
  G.cs = d; d += 64 * GM_MAXM;
  G.sn = d; d += 64 * GM_MAXM;
  G.y = d; d += 64 * GM_MAXM;
  G.hh = d; d += 64 * GB_Q;
  G.hh2 = d; d += 64 * GB_Q;
  G.H = d;
  HIPC(hipMemsetAsync(si.p, 0, sizeof(int) * (64 * 6 + 3 * 8), st));
  HIPC(hipMemsetAsync(sd.p, 0, sizeof(double) * 64 * 4, st));
  HIPC(hipMemcpyAsync(G.thr, thr, sizeof(double) * k, hipMemcpyHostToDevice, st));

  const double* Vb = basis.p;
  // the sparse products of the BiCGStab driver, on the columns whose flag is 0
  State Sarn{}, Scyc{};
  Sarn.status = G.arn;
  Sarn.skip = G.zero;
  Sarn.any = G.any_arn;
  Scyc.status = G.cyc;
  Scyc.skip = G.zero;
  Scyc.any = G.any_cyc;
  {
    const int ntk = tune_get("NT_STORE", -1);
    Sarn.nt = Scyc.nt = ntk >= 0 ? ntk : ((size_t)n * kp * sizeof(double) > (size_t(32) << 20) ? 1 : 0);
  }
  constexpr int RPB = (64 / LP) * (NT / 64);
  const int xmap = tune_get("XMAP", nk * sizeof(double) <= (size_t(256) << 20) ? 1 : 0);
  auto sp_grid = [&](const void* kern) {
    const int64_t ntiles = (n + RPB - 1) / RPB;
    int64_t g = std::min<int64_t>({(int64_t)NBMAX, ntiles, (int64_t)resident_blocks(kern, NT)});
    return (int)(g >= 8 ? (g & ~int64_t(7)) : g);
  };
  // the M product's gather batches follow the SPMM_M (SPMM_M_WIDE) knob, as in BiCGStab
  const int mvar = LP >= 32 ? tune_get("SPMM_M_WIDE", 4) : tune_get("SPMM_M", 1);
  const void* km = mvar == 0   ? (const void*)k_spmm<LP, TM, 8, 4>
                   : mvar == 2 ? (const void*)k_spmm<LP, TM, 5, 0>
                   : mvar == 3 ? (const void*)k_spmm<LP, TM, 16, 8>
                   : mvar == 4 ? (const void*)k_spmm<LP, TM, 2, 0>
                               : (const void*)k_spmm<LP, TM, 6, 3>;
  const void* ka = (const void*)k_spmm<LP, double, 6, 3>;
  const int gm = sp_grid(km), ga = sp_grid(ka);
  auto mprod = [&](const double* in, double* out, const State& S) {
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(gm), dim3(NT), 0, st, n, k, kp, M, in, out, S, xmap);
    };
    switch (mvar) {
      case 0: go(k_spmm<LP, TM, 8, 4>); break;
      case 2: go(k_spmm<LP, TM, 5, 0>); break;
      case 3: go(k_spmm<LP, TM, 16, 8>); break;
      case 4: go(k_spmm<LP, TM, 2, 0>); break;
      default: go(k_spmm<LP, TM, 6, 3>); break;
    }
  };
  auto aprod = [&](const double* in, double* out, const State& S) {
    hipLaunchKernelGGL((k_spmm<LP, double, 6, 3>), dim3(ga), dim3(NT), 0, st, n, k, kp, A, in, out, S, xmap);
  };
  const int rg = GB_RT / kp;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(GB_NB, (n + rg - 1) / rg));
  const unsigned eg = grid_for((int64_t)nk, GB_NT, 4096);
#define GB_CASES(X)                                                                              \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) \
  X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
  auto fin = [&](int nq, double* out) {
    hipLaunchKernelGGL(k_gb_fin, dim3(nq), dim3(GB_RT), 0, st, nb, kp, part.p, out);
  };
  // partials of V_{q0..q0+nv-1}^T W, nv <= GB_CH
  auto dots_chunk = [&](int q0, int nv, const double* W) {
    switch (nv) {
#define GB_X(N)                                                                                      \
  case N:                                                                                            \
    hipLaunchKernelGGL((k_gb_dots<N>), dim3(nb), dim3(GB_RT), 0, st, n, kp, q0, Vb, W, G.arn, G.any_arn, \
                       part.p);                                                                      \
    break;
      GB_CASES(GB_X)
#undef GB_X
    }
  };
  // W -= V_{q0..q0+nv-1} h[q0..], nv <= GB_CH (with the norm partials)
  auto project_chunk = [&](int q0, int nv, const double* h, double* W, int norm) {
    switch (nv) {
#define GB_X(N)                                                                                         \
  case N:                                                                                               \
    hipLaunchKernelGGL((k_gb_project<N>), dim3(nb), dim3(GB_RT), 0, st, n, kp, q0, Vb, h, W, G.arn, G.any_arn, \
                       norm, part.p);                                                                   \
    break;
      GB_CASES(GB_X)
#undef GB_X
    }
  };
  auto projdots = [&](int nv, const double* h, double* W) {
    switch (nv) {
#define GB_X(N)                                                                                          \
  case N:                                                                                                \
    hipLaunchKernelGGL((k_gb_projdots<N>), dim3(nb), dim3(GB_RT), 0, st, n, kp, Vb, h, W, G.arn, G.any_arn, \
                       part.p);                                                                          \
    break;
      GB_CASES(GB_X)
#undef GB_X
    }
  };
#undef GB_CASES
  // Gram-Schmidt twice against V_{0..nv-1}: hh, hh2 and nn = ||W||^2 after
  auto orthogonalise = [&](int nv, double* W) {
    for (int q0 = 0; q0 < nv; q0 += GB_CH) dots_chunk(q0, std::min(GB_CH, nv - q0), W);
    fin(nv, G.hh);
    if (nv <= GB_CH) {
      projdots(nv, G.hh, W);  // first projection fused with the second products
    } else {
      for (int q0 = 0; q0 < nv; q0 += GB_CH) project_chunk(q0, std::min(GB_CH, nv - q0), G.hh, W, 0);
      for (int q0 = 0; q0 < nv; q0 += GB_CH) dots_chunk(q0, std::min(GB_CH, nv - q0), W);
    }
    fin(nv, G.hh2);
    for (int q0 = 0; q0 < nv; q0 += GB_CH)
      project_chunk(q0, std::min(GB_CH, nv - q0), G.hh2, W, q0 + GB_CH >= nv ? 1 : 0);
    fin(1, G.nn);
  };

  HostStage hs(16);
  int* cnt = hs.as<int>();
  {
    SAI_PROF(GN.init, st);
    hipLaunchKernelGGL(k_gb_load, dim3(eg), dim3(GB_NT), 0, st, n, k, kp, R, Bv.p, Xv.p, Wv.p);
    // ||R|| per column (the "cycle" set is every column here)
    HIPC(hipMemsetAsync(G.any_cyc, 0xff, sizeof(int) * 8, st));
    hipLaunchKernelGGL(k_gb_resid, dim3(nb), dim3(GB_RT), 0, st, n, kp, Bv.p, Xv.p, Wv.p, G.zero, G.any_cyc,
                       part.p);
    fin(1, G.nn);
    hipLaunchKernelGGL(k_gb_setup, dim3(1), dim3(64), 0, st, k, maxit, G);
  }
  LAUNCH_CHECK();
  for (;;) {
    HIPC(hipMemcpyAsync(cnt, G.any_st + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (cnt[0] == 0) break;
    {
      SAI_PROF(GN.start, st);
      hipLaunchKernelGGL(k_gb_cycle_start, dim3(1), dim3(64), 0, st, k, m, G);
      hipLaunchKernelGGL(k_gb_scale, dim3(eg), dim3(GB_NT), 0, st, n, kp, G.a, Wv.p, basis.p, G.cyc,
                         G.any_cyc);
    }
    for (int j = 0; j < m; ++j) {
      {
        SAI_PROF(sizeof(TM) == 4 ? GN.m32 : GN.m64, st);
        mprod(Vb + nk * j, Zv.p, Sarn);
      }
      {
        SAI_PROF(GN.a, st);
        aprod(Zv.p, Wv.p, Sarn);
      }
      {
        SAI_PROF(GN.orth, st);
        orthogonalise(j + 1, Wv.p);
      }
      {
        SAI_PROF(GN.step, st);
        hipLaunchKernelGGL(k_gb_step, dim3(1), dim3(64), 0, st, k, m, j, maxit, G);
        if (j + 1 < m)
          hipLaunchKernelGGL(k_gb_scale, dim3(eg), dim3(GB_NT), 0, st, n, kp, G.a, Wv.p,
                             basis.p + nk * (j + 1), G.arn, G.any_arn);
      }
      LAUNCH_CHECK();
    }
    {
      SAI_PROF(GN.end, st);
      hipLaunchKernelGGL(k_gb_backsolve, dim3(1), dim3(64), 0, st, k, G);
      hipLaunchKernelGGL(k_gb_combine, dim3(eg), dim3(GB_NT), 0, st, n, kp, Vb, G.y, G.kk, Zv.p, G.cyc,
                         G.any_cyc);
      mprod(Zv.p, Wv.p, Scyc);
      hipLaunchKernelGGL(k_gb_add, dim3(eg), dim3(GB_NT), 0, st, n, kp, Wv.p, Xv.p, G.cyc, G.any_cyc);
      aprod(Xv.p, Zv.p, Scyc);
      hipLaunchKernelGGL(k_gb_resid, dim3(nb), dim3(GB_RT), 0, st, n, kp, Bv.p, Zv.p, Wv.p, G.cyc, G.any_cyc,
                         part.p);
      fin(1, G.nn);
      hipLaunchKernelGGL(k_gb_cycle_end, dim3(1), dim3(64), 0, st, k, maxit, G);
    }
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_gb_out, dim3(grid_for((int64_t)n * k, GB_NT, 4096)), dim3(GB_NT), 0, st, n, k, kp, Xv.p,
                     X);
  LAUNCH_CHECK();
  std::vector<int> hst(k), hit(k);
  HIPC(hipMemcpyAsync(hst.data(), G.st, sizeof(int) * k, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(hit.data(), G.it, sizeof(int) * k, hipMemcpyDeviceToHost, st));
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

#undef GB_COLS

template <class TM>
int gmres_batched(const Csr<double>& A, const Csr<TM>& M, int64_t n, int k, const double* R, double* X,
                  const double* thr, int m, int maxit, const Allocator& al, hipStream_t st, int* iters,
                  int* status, bool transposed) {
  switch (lp_class(k)) {
    case 1: return gmres_batched_lp<1, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    case 2: return gmres_batched_lp<2, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    case 4: return gmres_batched_lp<4, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    case 6: return gmres_batched_lp<6, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    case 8: return gmres_batched_lp<8, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    case 12: return gmres_batched_lp<12, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    case 16: return gmres_batched_lp<16, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
    default: return gmres_batched_lp<32, TM>(A, M, n, k, R, X, thr, m, maxit, al, st, iters, status, transposed);
  }
}

}  // namespace
}  // namespace sai
