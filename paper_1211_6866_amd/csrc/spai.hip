// SPAI adaptive pattern search on A~ (Section 2.1), in float64.
//
// From J = P(A~(:, k)), step 0 (the first solve and its residual test) runs
// for every column through the static pattern builder and the
// register-resident column solver; only the columns whose residual exceeds
// delta enter the search kernel (from {k}, every column does).  There one
// workgroup takes one column at a time from a counter, the largest step-0
// |I_k| first, and starting from J = P(A~(:, k)) (or {k}) runs each step:
//   I   = nonzero rows of A~(:, J)                         (gather, sort, unique)
//   m   = argmin ||A~(I, J) m - e_k(I)||                   (Householder QR)
//   r   = A~(:, J) m - e_k on I;  stop if ||r|| <= delta
//   N   = nonzero columns of A~(I, :);  J~ = N \ J         (candi)
//   g_j = (r^T A~ e_j)^2 / ||A~ e_j||^2 for j in J~        (from (muj), (rhoj):
//         rho_j^2 = ||r||^2 - g_j, so the largest g_j are the smallest rho_j)
//   J  += the per_step candidates of largest g_j (ties: smaller j).
// After at most `steps` augmentations the final J_k is written; the final
// least-squares solve in the build precision happens in the common column
// solver, as for the static patterns.  The candidate set is taken
// structurally (all rows of I_k).  Each augmentation updates the QR factors
// of the previous step (the rows the new columns bring are appended, the new
// columns reflected and factored), as Section 2.1 suggests.
#include "sai_internal.hpp"

#include <algorithm>

namespace sai {

void rows_of_patterns(const sai_split_s* sp, hipStream_t st, const Allocator& al,
                      const DBuf<int64_t>& jptr, const DBuf<int32_t>& jidx, DBuf<int64_t>& iptr,
                      DBuf<int32_t>& iidx, DBuf<int32_t>& cntI);
void build_patterns(const sai_split_s* sp, int kind, hipStream_t st, const Allocator& al,
                    DBuf<int64_t>& jptr, DBuf<int32_t>& jidx, DBuf<int64_t>& iptr,
                    DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ, DBuf<int32_t>& cntI);
template <class T>
int solve_columns(const sai_split_s* sp, const int64_t* jptr, const int32_t* jidx,
                  const int64_t* iptr, const int32_t* iidx, const int32_t* cntJ,
                  const int32_t* cntI, int maxI, int maxJ, T* mout, double* res,
                  int64_t* bucket_cols, const Allocator& al, hipStream_t st);

namespace {

constexpr int SNT = 256;
// Limits of one column's search workspace: |J_k| (J), |I_k| (I) and candidate or
// gathered entries before de-duplication (N, a power of two, at least 3 I).
// Every column is searched with the small limits first; a column that
// outgrows them is searched again from its start with the large ones, in a
// second launch with fewer, larger workspace slots.
template <int J_, int I_, int N_>
struct Caps {
  static constexpr int J = J_, I = I_, N = N_;
};
using CapS = Caps<128, 2048, 8192>;
using CapL = Caps<512, 8192, 65536>;
constexpr int SJMAX = CapS::J;   // |J_k| of the padded per-column result arrays
constexpr int NSLOT_MAX = 4096;  // columns searched concurrently (workspace slots), at most
constexpr int NSLOT_L = 64;      // ... with the large limits
// result of a column solve: done, over the workspace limits, rank deficient
enum { LS_OK = 0, LS_BIG = 1, LS_SING = 2 };

enum { E_TOOBIG = 1, E_SING = 2 };

struct Ws {
  int32_t* I;     // C::I
  int32_t* cand;  // C::N
  int32_t* off;   // C::I + 1
  double* W;      // C::I * (C::J + 1), column-major block + right-hand side
  double* r;      // C::I
  double* g;      // C::N
  int32_t* Is;    // C::I, SPAI search only: I sorted
  int32_t* P;     // C::I, SPAI search only: storage row of Is[q]
};

__device__ __forceinline__ int bsearch_eq(const int32_t* a, int n, int32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return (lo < n && a[lo] == x) ? lo : -1;
}

template <int B>
__device__ double blk_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < B / WAVE; ++i) s += red[i];
  __syncthreads();
  return s;
}

// In-place exclusive prefix sum of a[0..m); returns the total.
template <int B>
__device__ int blk_exscan(int32_t* a, int m, int* wsum /* B/WAVE + 1 */) {
  const int tid = threadIdx.x, w = tid / WAVE, l = tid % WAVE;
  int carry = 0;
  for (int base = 0; base < m; base += B) {
    const int i = base + tid;
    const int v = i < m ? a[i] : 0;
    int incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int t = __shfl_up(incl, o, WAVE);
      if (l >= o) incl += t;
    }
    __syncthreads();
    if (l == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int q = 0; q < B / WAVE; ++q) {
      if (q < w) woff += wsum[q];
      tot += wsum[q];
    }
    if (i < m) a[i] = carry + woff + incl - v;
    carry += tot;
    __syncthreads();
  }
  return carry;
}

// Keep a[i] where keep(i) holds, preserving order (in place); returns the count.
template <int B, class Pred>
__device__ int blk_compact(int32_t* a, int m, Pred keep, int* wsum) {
  const int tid = threadIdx.x, w = tid / WAVE, l = tid % WAVE;
  int out = 0;
  for (int base = 0; base < m; base += B) {
    const int i = base + tid;
    int32_t v = 0;
    bool k = false;
    if (i < m) {
      v = a[i];
      k = keep(i, v);
    }
    const unsigned long long bal = __ballot(k);
    const int before = __popcll(bal & ((l == 0) ? 0ull : (~0ull >> (64 - l))));
    __syncthreads();
    if (l == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int woff = 0, tot = 0;
    for (int q = 0; q < B / WAVE; ++q) {
      if (q < w) woff += wsum[q];
      tot += wsum[q];
    }
    if (k) a[out + woff + before] = v;
    out += tot;
    __syncthreads();
  }
  return out;
}

// Bitonic sort of a[0..m) (padded to a power of two <= cap) and de-duplication.
template <int B>
__device__ int blk_sort_unique(int32_t* a, int m, int* wsum) {
  const int tid = threadIdx.x;
  int P = 1;
  while (P < m) P <<= 1;
  for (int i = m + tid; i < P; i += B) a[i] = 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = tid; t < (P >> 1); t += B) {
        const int i = 2 * j * (t / j) + (t % j);
        const int q = i + j;
        const int32_t x = a[i], y = a[q];
        if ((x > y) == ((i & k) == 0)) { a[i] = y; a[q] = x; }
      }
      __syncthreads();
    }
  }
  // the predicate reads the sorted array before any write of this chunk
  return blk_compact<B>(a, m, [&](int i, int32_t v) { return i == 0 || a[i - 1] != v; }, wsum);
}

__global__ void __launch_bounds__(SNT) k_colnorm2(int32_t n, const int32_t* cp, const double* cv,
                                                  double* out) {
  const int64_t j = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int32_t e = cp[j]; e < cp[j + 1]; ++e) s += cv[e] * cv[e];
  out[j] = s;
}

// Least-squares solve of column k on the pattern sJ[0..nJ) in the workgroup's
// workspace: I = nonzero rows of A~(:, J) (ws.I, sorted), the dense block
// A~(I, J) with e_k(I) (ws.W), Householder QR with Q^T applied to e_k,
// back-substitution into sm[0..nJ), and the residual r = A~(:, J) m - e_k on I
// (ws.r, columns added in order).  Returns LS_BIG when |I| or the gathered
// entries exceed the workspace limits C, LS_SING when the block is rank
// deficient (the same in every thread); rr = ||r||^2.  Every thread of the
// workgroup calls it.
template <int B, class C>
__device__ int ls_solve_ws(int64_t k, const int32_t* __restrict__ cp, const int32_t* __restrict__ ri,
                            const double* __restrict__ cv, const int32_t* sJ, int nJ, const Ws& ws,
                            double* sm, double* sd, double* red, int* wsum, int* s_int, int& nI_out,
                            double& rr) {
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  // ---- I = rows of A~(:, J)
  int tot = 0;
  if (tid == 0) {
    int acc = 0;
    for (int c = 0; c < nJ; ++c) {
      ws.off[c] = acc;
      acc += cp[sJ[c] + 1] - cp[sJ[c]];
    }
    ws.off[nJ] = acc;
    s_int[0] = acc;
  }
  __syncthreads();
  tot = s_int[0];
  if (tot > C::N) return LS_BIG;
  for (int f = tid; f < tot; f += B) {
    int lo = 0, hi = nJ - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ws.off[mid] <= f) lo = mid; else hi = mid - 1;
    }
    ws.cand[f] = ri[cp[sJ[lo]] + (f - ws.off[lo])];
  }
  __syncthreads();
  const int nI = blk_sort_unique<B>(ws.cand, tot, wsum);
  if (nI > C::I) return LS_BIG;
  if (nI < nJ) return LS_SING;
  for (int t = tid; t < nI; t += B) ws.I[t] = ws.cand[t];
  __syncthreads();
  // ---- dense block A~(I, J) (column-major, ld nI) and e_k(I) in column nJ
  double* W = ws.W;
  double* bv = W + (int64_t)nI * nJ;
  for (int64_t t = tid; t < (int64_t)nI * (nJ + 1); t += B) W[t] = 0.0;
  __syncthreads();
  for (int c = 0; c < nJ; ++c) {
    const int32_t j = sJ[c];
    for (int32_t e = cp[j] + tid; e < cp[j + 1]; e += B) {
      const int pos = bsearch_eq(ws.I, nI, ri[e]);
      W[(int64_t)c * nI + pos] = cv[e];
    }
  }
  for (int t = tid; t < nI; t += B) bv[t] = (ws.I[t] == k) ? 1.0 : 0.0;
  __syncthreads();
  // ---- Householder QR, Q^T applied to the right-hand side
  bool sing = false;
  for (int j = 0; j < nJ; ++j) {
    double* colj = W + (int64_t)j * nI;
    double tail = 0.0;
    for (int t = j + 1 + tid; t < nI; t += B) tail += colj[t] * colj[t];
    tail = blk_sum<B>(tail, red);
    const double alpha = colj[j];
    const double normx = sqrt(tail + alpha * alpha);
    const double sgn = alpha >= 0.0 ? 1.0 : -1.0;
    const double vj = alpha + sgn * normx;
    const double vtv = tail + vj * vj;
    if (!(normx > 0.0)) sing = true;
    const double tau = normx > 0.0 ? 2.0 / vtv : 0.0;
    __syncthreads();
    if (tid == 0) colj[j] = vj;
    __syncthreads();
    for (int c = j + 1 + w; c <= nJ; c += B / WAVE) {
      const double* colc = W + (int64_t)c * nI;
      double d = 0.0;
      for (int t = j + lane; t < nI; t += WAVE) d += colj[t] * colc[t];
      d = wave_sum(d);
      if (lane == 0) sd[c] = tau * d;
    }
    __syncthreads();
    const int rows = nI - j, ncol = nJ - j;
    for (int64_t t = tid; t < (int64_t)rows * ncol; t += B) {
      const int c = j + 1 + (int)(t / rows);
      const int rr = j + (int)(t % rows);
      W[(int64_t)c * nI + rr] -= sd[c] * colj[rr];
    }
    __syncthreads();
    if (tid == 0) colj[j] = -sgn * normx;
    __syncthreads();
  }
  if (sing) return LS_SING;
  if (w == 0) {
    for (int c = nJ - 1; c >= 0; --c) {
      double part = 0.0;
      for (int q = c + 1 + lane; q < nJ; q += WAVE) part += W[(int64_t)q * nI + c] * sm[q];
      part = wave_sum(part);
      if (lane == 0) sm[c] = (bv[c] - part) / W[(int64_t)c * nI + c];
    }
  }
  __syncthreads();
  // ---- residual r = A~(:, J) m - e_k on I (columns added in order)
  for (int t = tid; t < nI; t += B) ws.r[t] = (ws.I[t] == k) ? -1.0 : 0.0;
  __syncthreads();
  for (int c = 0; c < nJ; ++c) {
    const int32_t j = sJ[c];
    const double mc = sm[c];
    for (int32_t e = cp[j] + tid; e < cp[j + 1]; e += B) {
      const int pos = bsearch_eq(ws.I, nI, ri[e]);
      ws.r[pos] += cv[e] * mc;
    }
    __syncthreads();
  }
  rr = 0.0;
  for (int t = tid; t < nI; t += B) rr += ws.r[t] * ws.r[t];
  rr = blk_sum<B>(rr, red);
  nI_out = nI;
  return LS_OK;
}

// Least-squares solve of the SPAI search with its QR factors updated as J
// grows (Section 2.1 notes that the factors of the augmented problem follow
// from the previous ones).  State kept in the workspace between calls:
//   ws.I[0..nI)   rows of I_k in storage order (the rows a step adds go last),
//   ws.Is[0..nI)  the same rows sorted, ws.P[q] = storage row of ws.Is[q],
//   ws.W          factor column c at W + c * C::I: R above the diagonal, the
//                 reflector's other entries below it; Q^T e_k(I) at W + C::J * C::I,
//   hv[c], ht[c]  leading entry and coefficient 2 / (v^T v) of reflector c.
// Columns fJ[0..j0) are factored; this call adds fJ[j0..nJ): it gathers the
// rows they bring, applies the stored reflectors to the new columns, factors
// them, and back-substitutes into sm[0..nJ) (factor order).  Old columns and
// reflectors are zero in the new rows, so the factors are those of the
// row-permuted block A~(I, J) and the minimiser is the same as a solve from
// scratch.  r = A~(:, J) m - e_k on I goes to ws.r (storage order, columns
// added in factor order), rr = ||r||^2.  Returns LS_BIG (the same in every
// thread) when the workspace would overflow, LS_SING when a new column is
// dependent.
template <int B, class C>
__device__ int ls_extend_ws(int64_t k, const int32_t* __restrict__ cp, const int32_t* __restrict__ ri,
                             const double* __restrict__ cv, const int32_t* fJ, int j0, int nJ,
                             const Ws& ws, double* sm, double* sd, double* hv, double* ht, double* red,
                             int* wsum, int* s_int, int& nI, double& rr) {
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int nI0 = nI;
  // ---- rows of the new columns that are not yet in I
  if (tid == 0) {
    int acc = 0;
    for (int c = j0; c < nJ; ++c) {
      ws.off[c - j0] = acc;
      acc += cp[fJ[c] + 1] - cp[fJ[c]];
    }
    ws.off[nJ - j0] = acc;
    s_int[0] = acc;
  }
  __syncthreads();
  const int tot = s_int[0];
  if (tot > C::N) return LS_BIG;
  for (int f = tid; f < tot; f += B) {
    int lo = 0, hi = nJ - j0 - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ws.off[mid] <= f) lo = mid; else hi = mid - 1;
    }
    ws.cand[f] = ri[cp[fJ[j0 + lo]] + (f - ws.off[lo])];
  }
  __syncthreads();
  int nNew = blk_sort_unique<B>(ws.cand, tot, wsum);
  nNew = blk_compact<B>(ws.cand, nNew, [&](int, int32_t v) { return bsearch_eq(ws.Is, nI0, v) < 0; }, wsum);
  const int nI1 = nI0 + nNew;
  if (nI1 > C::I) return LS_BIG;
  if (nI1 < nJ) return LS_SING;
  // ---- merge the new rows into the sorted copy (cand + C::I / + 2 C::I as staging)
  int32_t* tS = ws.cand + C::I;
  int32_t* tP = ws.cand + 2 * C::I;
  for (int q = tid; q < nI0; q += B) {
    const int32_t v = ws.Is[q];
    int lo = 0, hi = nNew;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ws.cand[mid] < v) lo = mid + 1; else hi = mid;
    }
    tS[q + lo] = v;
    tP[q + lo] = ws.P[q];
  }
  for (int q = tid; q < nNew; q += B) {
    const int32_t v = ws.cand[q];
    int lo = 0, hi = nI0;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ws.Is[mid] < v) lo = mid + 1; else hi = mid;
    }
    tS[q + lo] = v;
    tP[q + lo] = nI0 + q;
    ws.I[nI0 + q] = v;
  }
  __syncthreads();
  for (int q = tid; q < nI1; q += B) {
    ws.Is[q] = tS[q];
    ws.P[q] = tP[q];
  }
  // ---- new rows of the factored columns are zero; e_k on the new rows; the new columns
  double* W = ws.W;
  double* bv = W + (int64_t)C::J * C::I;
  for (int t = tid; t < j0 * nNew; t += B) W[(int64_t)(t / nNew) * C::I + nI0 + t % nNew] = 0.0;
  for (int t = tid; t < nNew; t += B) bv[nI0 + t] = (ws.I[nI0 + t] == k) ? 1.0 : 0.0;
  for (int t = tid; t < (nJ - j0) * nI1; t += B) W[(int64_t)(j0 + t / nI1) * C::I + t % nI1] = 0.0;
  __syncthreads();
  for (int c = j0; c < nJ; ++c) {
    const int32_t j = fJ[c];
    for (int32_t e = cp[j] + tid; e < cp[j + 1]; e += B) {
      const int q = bsearch_eq(ws.Is, nI1, ri[e]);
      W[(int64_t)c * C::I + ws.P[q]] = cv[e];
    }
  }
  __syncthreads();
  // ---- stored reflectors applied to the new columns: one wavefront per column,
  // storage row t always handled by lane t % WAVE
  for (int c = j0 + w; c < nJ; c += B / WAVE) {
    double* colc = W + (int64_t)c * C::I;
    for (int j = 0; j < j0; ++j) {
      const double* colj = W + (int64_t)j * C::I;
      double d = 0.0;
      for (int t = lane; t < nI1; t += WAVE) {
        if (t > j) d += colj[t] * colc[t];
        else if (t == j) d += hv[j] * colc[t];
      }
      d = ht[j] * wave_sum(d);
      for (int t = lane; t < nI1; t += WAVE) {
        if (t > j) colc[t] -= d * colj[t];
        else if (t == j) colc[t] -= d * hv[j];
      }
    }
  }
  __syncthreads();
  // ---- Householder steps on the new columns, applied to the later ones and Q^T e_k
  bool sing = false;
  for (int j = j0; j < nJ; ++j) {
    double* colj = W + (int64_t)j * C::I;
    double tail = 0.0;
    for (int t = j + 1 + tid; t < nI1; t += B) tail += colj[t] * colj[t];
    tail = blk_sum<B>(tail, red);
    const double alpha = colj[j];
    const double normx = sqrt(tail + alpha * alpha);
    const double sgn = alpha >= 0.0 ? 1.0 : -1.0;
    const double vj = alpha + sgn * normx;
    const double vtv = tail + vj * vj;
    if (!(normx > 0.0)) sing = true;
    const double tau = normx > 0.0 ? 2.0 / vtv : 0.0;
    __syncthreads();
    if (tid == 0) {
      colj[j] = vj;
      hv[j] = vj;
      ht[j] = tau;
    }
    __syncthreads();
    for (int c = j + 1 + w; c <= nJ; c += B / WAVE) {
      const double* colc = c == nJ ? bv : W + (int64_t)c * C::I;
      double d = 0.0;
      for (int t = j + lane; t < nI1; t += WAVE) d += colj[t] * colc[t];
      d = wave_sum(d);
      if (lane == 0) sd[c] = tau * d;
    }
    __syncthreads();
    const int rows = nI1 - j, ncol = nJ - j;
    for (int64_t t = tid; t < (int64_t)rows * ncol; t += B) {
      const int c = j + 1 + (int)(t / rows);
      const int r_ = j + (int)(t % rows);
      double* colc = c == nJ ? bv : W + (int64_t)c * C::I;
      colc[r_] -= sd[c] * colj[r_];
    }
    __syncthreads();
    if (tid == 0) colj[j] = -sgn * normx;
    __syncthreads();
  }
  if (sing) return LS_SING;
  if (w == 0) {
    for (int c = nJ - 1; c >= 0; --c) {
      double part = 0.0;
      for (int q = c + 1 + lane; q < nJ; q += WAVE) part += W[(int64_t)q * C::I + c] * sm[q];
      part = wave_sum(part);
      if (lane == 0) sm[c] = (bv[c] - part) / W[(int64_t)c * C::I + c];
    }
  }
  __syncthreads();
  // ---- residual r = A~(:, J) m - e_k on I
  for (int t = tid; t < nI1; t += B) ws.r[t] = (ws.I[t] == k) ? -1.0 : 0.0;
  __syncthreads();
  for (int c = 0; c < nJ; ++c) {
    const int32_t j = fJ[c];
    const double mc = sm[c];
    for (int32_t e = cp[j] + tid; e < cp[j + 1]; e += B) {
      const int q = bsearch_eq(ws.Is, nI1, ri[e]);
      ws.r[ws.P[q]] += cv[e] * mc;
    }
    __syncthreads();
  }
  rr = 0.0;
  for (int t = tid; t < nI1; t += B) rr += ws.r[t] * ws.r[t];
  rr = blk_sum<B>(rr, red);
  nI = nI1;
  return LS_OK;
}

// A column the workspace limits C cannot hold is appended to ovf (when given:
// it is searched again with the large limits), else it is an error.
template <int B, class C>
__global__ void __launch_bounds__(B) k_spai(int32_t n, const int32_t* __restrict__ cp,
                                              const int32_t* __restrict__ ri,
                                              const double* __restrict__ cv,
                                              const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci,
                                              const double* __restrict__ cn2, int steps, int per,
                                              double delta, int init,
                                              const int64_t* __restrict__ jpoff,
                                              int32_t* __restrict__ jpad, int32_t* __restrict__ cntJ,
                                              Ws ws0, const int32_t* __restrict__ list, int32_t nwork,
                                              int* __restrict__ next, int* __restrict__ err,
                                              int32_t* __restrict__ taken, int32_t* __restrict__ ovf,
                                              int* __restrict__ ovf_cnt) {
  __shared__ int32_t sJ[C::J + 8];
  __shared__ int32_t fJ[C::J];
  __shared__ double sm[C::J];
  __shared__ double sd[C::J + 1];
  __shared__ double hv[C::J];
  __shared__ double ht[C::J];
  __shared__ double red[B / WAVE];
  __shared__ int wsum[B / WAVE + 1];
  __shared__ int32_t chosen[16];
  __shared__ int s_int[4];
  __shared__ int s_it;
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int slot = blockIdx.x;
  Ws ws;
  ws.I = ws0.I + (int64_t)slot * C::I;
  ws.cand = ws0.cand + (int64_t)slot * C::N;
  ws.off = ws0.off + (int64_t)slot * (C::I + 1);
  ws.W = ws0.W + (int64_t)slot * C::I * (C::J + 1);
  ws.r = ws0.r + (int64_t)slot * C::I;
  ws.g = ws0.g + (int64_t)slot * C::N;
  ws.Is = ws0.Is + (int64_t)slot * C::I;
  ws.P = ws0.P + (int64_t)slot * C::I;

  // columns are taken one at a time from the counter `next` (the list holds
  // the costly ones first), so that no workgroup is left with a queue of them
  for (;;) {
    __syncthreads();  // every thread has read the previous s_it
    if (tid == 0) s_it = atomicAdd(next, 1);
    __syncthreads();
    const int it = s_it;
    if (it >= nwork) break;
    const int64_t k = list ? list[it] : it;
    // ---- initial pattern
    int nJ;
    int fcode = LS_OK;
    if (init == SAI_INIT_DIAG) {
      if (tid == 0) sJ[0] = fJ[0] = (int32_t)k;
      nJ = 1;
    } else {
      nJ = cp[k + 1] - cp[k];
      if (nJ > C::J) fcode = LS_BIG;
      else
        for (int t = tid; t < nJ; t += B) sJ[t] = fJ[t] = ri[cp[k] + t];
    }
    __syncthreads();
    int nI = 0, j0 = 0, naug = 0;
    for (int step = 0; step < steps && fcode == LS_OK; ++step) {
      double rr = 0.0;
      fcode = ls_extend_ws<B, C>(k, cp, ri, cv, fJ, j0, nJ, ws, sm, sd, hv, ht, red, wsum, s_int, nI, rr);
      if (fcode != LS_OK) break;
      j0 = nJ;
      if (sqrt(rr) <= delta) break;
      // ---- candidates: nonzero columns of A~(I, :), minus J
      for (int t = tid; t < nI; t += B) ws.off[t] = rp[ws.I[t] + 1] - rp[ws.I[t]];
      __syncthreads();
      const int ntot = blk_exscan<B>(ws.off, nI, wsum);
      if (tid == 0) ws.off[nI] = ntot;
      __syncthreads();
      if (ntot > C::N) { fcode = LS_BIG; break; }
      for (int f = tid; f < ntot; f += B) {
        int lo = 0, hi = nI - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (ws.off[mid] <= f) lo = mid; else hi = mid - 1;
        }
        ws.cand[f] = ci[rp[ws.I[lo]] + (f - ws.off[lo])];
      }
      __syncthreads();
      int nN = blk_sort_unique<B>(ws.cand, ntot, wsum);
      nN = blk_compact<B>(ws.cand, nN, [&](int, int32_t v) { return bsearch_eq(sJ, nJ, v) < 0; }, wsum);
      if (nN == 0) break;
      // ---- gains g_j = (r^T A~ e_j)^2 / ||A~ e_j||^2
      for (int t = tid; t < nN; t += B) {
        const int32_t j = ws.cand[t];
        double tj = 0.0;
        for (int32_t e = cp[j]; e < cp[j + 1]; ++e) {
          const int q = bsearch_eq(ws.Is, nI, ri[e]);
          if (q >= 0) tj += ws.r[ws.P[q]] * cv[e];
        }
        ws.g[t] = tj * tj / cn2[j];
      }
      __syncthreads();
      // ---- the `add` largest gains, ties to the smaller column index
      const int add = min(per, nN);
      if (nJ + add > C::J) { fcode = LS_BIG; break; }
      for (int q = 0; q < add; ++q) {
        double bg = -1.0;
        int bt = -1;
        for (int t = tid; t < nN; t += B) {
          const double gv = ws.g[t];
          if (gv > bg || (gv == bg && bt >= 0 && ws.cand[t] < ws.cand[bt])) { bg = gv; bt = t; }
        }
        // wave argmax, then across waves
        for (int o = WAVE / 2; o > 0; o >>= 1) {
          const double og = __shfl_xor(bg, o, WAVE);
          const int ot = __shfl_xor(bt, o, WAVE);
          const bool better = ot >= 0 && (og > bg || (og == bg && (bt < 0 || ws.cand[ot] < ws.cand[bt])));
          if (better) { bg = og; bt = ot; }
        }
        __syncthreads();
        if (lane == 0) { red[w] = bg; wsum[w] = bt; }
        __syncthreads();
        if (tid == 0) {
          double gbest = -1.0;
          int tbest = -1;
          for (int q2 = 0; q2 < B / WAVE; ++q2) {
            const double og = red[q2];
            const int ot = wsum[q2];
            if (ot >= 0 && (og > gbest || (og == gbest && (tbest < 0 || ws.cand[ot] < ws.cand[tbest])))) {
              gbest = og;
              tbest = ot;
            }
          }
          chosen[q] = ws.cand[tbest];
          ws.g[tbest] = -2.0;  // taken
        }
        __syncthreads();
      }
      // ---- J = sorted(J + chosen); the factor order appends them
      if (tid == 0) {
        for (int q = 0; q < add; ++q) {
          const int32_t v = chosen[q];
          fJ[nJ] = v;
          int pos = nJ;
          while (pos > 0 && sJ[pos - 1] > v) {
            sJ[pos] = sJ[pos - 1];
            --pos;
          }
          sJ[pos] = v;
          ++nJ;
        }
        s_int[1] = nJ;
      }
      __syncthreads();
      nJ = s_int[1];
      ++naug;
    }
    if (fcode != LS_OK) {
      if (tid == 0) {
        if (fcode == LS_SING) atomicOr(err, E_SING);
        else if (ovf) ovf[atomicAdd(ovf_cnt, 1)] = (int32_t)k;
        else atomicOr(err, E_TOOBIG);
      }
      __syncthreads();
      continue;
    }
    const int64_t o = jpoff[k];
    for (int t = tid; t < nJ; t += B) jpad[o + t] = sJ[t];
    if (tid == 0) {
      cntJ[k] = nJ;
      taken[k] = naug;
    }
    __syncthreads();
  }
}

// PSAI(tol) (Section 2.2) on A~, in float64, one workgroup per column.  From
// S = F = {k} (a^(0) = e_k), loop l = 0 .. lmax:
//   F = nonzero rows of A~(:, F)       (P(a^(l+1)), structural)
//   S = S u F
//   m = argmin ||A~(I, S) m - e_k(I)||, r = A~(:, S) m - e_k   (lsprob)
//   drop |m_j| <= delta / (|S| ||A~||_1), the largest entry kept (first of
//   equals)                                                    (tolk)
//   stop when ||r|| <= delta (the residual before the drop).
// The kept entries keep their values (no re-solve).  The final S and m go to
// jpad / mpad at k * C::J (or, with out_list, at the work item's position
// times C::J), |S| to cntJ[k], ||r|| to res[k].  A column the limits C cannot
// hold is appended to ovf (when given), else it is an error.
template <int B, class C>
__global__ void __launch_bounds__(B) k_psai(int32_t n, const int32_t* __restrict__ cp,
                                              const int32_t* __restrict__ ri,
                                              const double* __restrict__ cv, int lmax, double delta,
                                              double a1, int32_t* __restrict__ jpad,
                                              double* __restrict__ mpad, int32_t* __restrict__ cntJ,
                                              double* __restrict__ res, Ws ws0,
                                              int32_t* __restrict__ fr0, const int32_t* __restrict__ list,
                                              int32_t nwork, int* __restrict__ err,
                                              int32_t* __restrict__ loops, int out_list,
                                              int32_t* __restrict__ ovf, int* __restrict__ ovf_cnt) {
  __shared__ int32_t sJ[C::J + 8];
  __shared__ double sm[C::J];
  __shared__ double sd[C::J + 1];
  __shared__ double red[B / WAVE];
  __shared__ int wsum[B / WAVE + 1];
  __shared__ int s_int[4];
  const int tid = threadIdx.x;
  const int slot = blockIdx.x;
  Ws ws;
  ws.I = ws0.I + (int64_t)slot * C::I;
  ws.cand = ws0.cand + (int64_t)slot * C::N;
  ws.off = ws0.off + (int64_t)slot * (C::I + 1);
  ws.W = ws0.W + (int64_t)slot * C::I * (C::J + 1);
  ws.r = ws0.r + (int64_t)slot * C::I;
  ws.g = ws0.g + (int64_t)slot * C::N;
  int32_t* F = fr0 + (int64_t)slot * C::I;  // P(a^(l)), sorted

  // work item b is column list[b] (or column b when list is NULL)
  for (int64_t b = blockIdx.x; b < nwork; b += gridDim.x) {
    const int64_t k = list ? (int64_t)list[b] : b;
    if (tid == 0) {
      sJ[0] = (int32_t)k;
      F[0] = (int32_t)k;
    }
    int nJ = 1, nF = 1;
    __syncthreads();
    int fcode = LS_OK;
    double rr = 0.0;
    int used = 0;
    for (int l = 0; l <= lmax; ++l) {
      used = l + 1;
      // ---- F = nonzero rows of A~(:, F)
      for (int t = tid; t < nF; t += B) ws.off[t] = cp[F[t] + 1] - cp[F[t]];
      __syncthreads();
      const int tot = blk_exscan<B>(ws.off, nF, wsum);
      if (tid == 0) ws.off[nF] = tot;
      __syncthreads();
      if (tot > C::N) { fcode = LS_BIG; break; }
      for (int f = tid; f < tot; f += B) {
        int lo = 0, hi = nF - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (ws.off[mid] <= f) lo = mid; else hi = mid - 1;
        }
        ws.cand[f] = ri[cp[F[lo]] + (f - ws.off[lo])];
      }
      __syncthreads();
      nF = blk_sort_unique<B>(ws.cand, tot, wsum);
      if (nF > C::I) { fcode = LS_BIG; break; }
      for (int t = tid; t < nF; t += B) F[t] = ws.cand[t];
      __syncthreads();
      // ---- S = S u F
      for (int t = tid; t < nF; t += B) ws.cand[t] = F[t];
      for (int t = tid; t < nJ; t += B) ws.cand[nF + t] = sJ[t];
      __syncthreads();
      const int nS = blk_sort_unique<B>(ws.cand, nF + nJ, wsum);
      if (nS > C::J) { fcode = LS_BIG; break; }
      for (int t = tid; t < nS; t += B) sJ[t] = ws.cand[t];
      nJ = nS;
      __syncthreads();
      // ---- least-squares solve on S
      int nI = 0;
      fcode = ls_solve_ws<B, C>(k, cp, ri, cv, sJ, nJ, ws, sm, sd, red, wsum, s_int, nI, rr);
      if (fcode != LS_OK) break;
      // ---- (tolk) drop, the largest entry (first of equals) kept
      if (tid == 0) {
        const double tol = delta / ((double)nJ * a1);
        int big = 0;
        for (int c = 1; c < nJ; ++c)
          if (fabs(sm[c]) > fabs(sm[big])) big = c;
        int q = 0;
        for (int c = 0; c < nJ; ++c) {
          if (fabs(sm[c]) > tol || c == big) {
            sJ[q] = sJ[c];
            sm[q] = sm[c];
            ++q;
          }
        }
        s_int[1] = q;
      }
      __syncthreads();
      nJ = s_int[1];
      if (sqrt(rr) <= delta) break;
    }
    if (fcode != LS_OK) {
      if (tid == 0) {
        if (fcode == LS_SING) atomicOr(err, E_SING);
        else if (ovf) ovf[atomicAdd(ovf_cnt, 1)] = (int32_t)k;
        else atomicOr(err, E_TOOBIG);
      }
      __syncthreads();
      continue;
    }
    const int64_t o = (out_list ? b : k) * C::J;
    for (int t = tid; t < nJ; t += B) {
      jpad[o + t] = sJ[t];
      mpad[o + t] = sm[t];
    }
    if (tid == 0) {
      cntJ[k] = nJ;
      res[k] = sqrt(rr);
      loops[k] = used;
    }
    __syncthreads();
  }
}

// PSAI(tol) loop l = 0 from a solve on J_k = P(A~(:, k)), which is S^(1) =
// P(A~ e_k) u {k} when the column holds its diagonal: the (tolk) drop, and the
// column is finished when ||r|| <= delta or lmax = 0 (its kept entries go to
// jpad / mpad at k * SJMAX); otherwise, or without a diagonal, todo[k] = 1 and
// the search kernel redoes it from loop 0.  One thread per column.
__global__ void __launch_bounds__(SNT) k_psai_first(int32_t n, const int64_t* __restrict__ jptr,
                                                    const int32_t* __restrict__ jidx,
                                                    const double* __restrict__ m,
                                                    const double* __restrict__ r, double delta,
                                                    double a1, int lmax, int32_t* __restrict__ jpad,
                                                    double* __restrict__ mpad, int32_t* __restrict__ cntJ,
                                                    double* __restrict__ res, int32_t* __restrict__ todo,
                                                    int32_t* __restrict__ loops) {
  const int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (k >= n) return;
  const int64_t a = jptr[k];
  const int nJ = (int)(jptr[k + 1] - a);
  bool diag = false;
  for (int c = 0; c < nJ; ++c) diag |= jidx[a + c] == (int32_t)k;
  if (!diag || nJ > SJMAX || !(r[k] <= delta || lmax == 0)) {
    todo[k] = 1;
    return;
  }
  todo[k] = 0;
  const double tol = delta / ((double)nJ * a1);
  int big = 0;
  for (int c = 1; c < nJ; ++c)
    if (fabs(m[a + c]) > fabs(m[a + big])) big = c;
  int q = 0;
  for (int c = 0; c < nJ; ++c) {
    if (fabs(m[a + c]) > tol || c == big) {
      jpad[k * SJMAX + q] = jidx[a + c];
      mpad[k * SJMAX + q] = m[a + c];
      ++q;
    }
  }
  cntJ[k] = q;
  res[k] = r[k];
  loops[k] = 1;
}

// out[0] = max cntI, out[1] = max cntJ (block maxima, one atomic per block)
__global__ void __launch_bounds__(SNT) k_max2(int32_t n, const int32_t* __restrict__ cntI,
                                              const int32_t* __restrict__ cntJ, int* __restrict__ out) {
  __shared__ int red[2][SNT / WAVE];
  int mi = 0, mj = 0;
  for (int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x; k < n; k += (int64_t)gridDim.x * SNT) {
    mi = max(mi, cntI[k]);
    mj = max(mj, cntJ[k]);
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    mi = max(mi, __shfl_xor(mi, o, WAVE));
    mj = max(mj, __shfl_xor(mj, o, WAVE));
  }
  if (threadIdx.x % WAVE == 0) {
    red[0][threadIdx.x / WAVE] = mi;
    red[1][threadIdx.x / WAVE] = mj;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < SNT / WAVE; ++q) {
      mi = max(mi, red[0][q]);
      mj = max(mj, red[1][q]);
    }
    atomicMax(&out[0], mi);
    atomicMax(&out[1], mj);
  }
}

// The columns with flag[k] != 0, in unspecified order (at most cap kept), and their number.
__global__ void __launch_bounds__(SNT) k_list_flagged(int32_t n, const int32_t* __restrict__ flag,
                                                      int32_t* __restrict__ list, int cap,
                                                      int* __restrict__ count) {
  const int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x;
  const bool f = k < n && flag[k] != 0;
  const int slot = block_slot<1>(count, f ? 0 : -1);
  if (f && slot < cap) list[slot] = (int32_t)k;
}

__global__ void __launch_bounds__(SNT) k_gather_i32(int32_t m, const int32_t* __restrict__ idx,
                                                    const int32_t* __restrict__ src,
                                                    int32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (t < m) out[t] = src[idx[t]];
}

__global__ void __launch_bounds__(SNT) k_colabs(int32_t n, const int32_t* cp, const double* cv,
                                                double* out) {
  const int64_t j = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int32_t e = cp[j]; e < cp[j + 1]; ++e) s += fabs(cv[e]);
  out[j] = s;
}

// Copy the padded rows (k * SJMAX, length cnt[k]) of a list and its values to
// their packed offsets off[k]; a column searched with the large limits
// (bigpos[k] = q >= 0) is read from row q of bigJ / bigM (stride CapL::J).
__global__ void k_compact_psai(int32_t n, const int32_t* __restrict__ jpad,
                               const double* __restrict__ mpad, const int64_t* __restrict__ off,
                               int32_t* __restrict__ jout, double* __restrict__ mout,
                               const int32_t* __restrict__ bigpos, const int32_t* __restrict__ bigJ,
                               const double* __restrict__ bigM) {
  const int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (k >= n) return;
  const int64_t a = off[k], b = off[k + 1];
  const int32_t q = bigpos ? bigpos[k] : -1;
  const int32_t* js = q >= 0 ? bigJ + (int64_t)q * CapL::J : jpad + k * SJMAX;
  const double* ms = q >= 0 ? bigM + (int64_t)q * CapL::J : mpad + k * SJMAX;
  for (int64_t t = 0; t < b - a; ++t) {
    jout[a + t] = js[t];
    mout[a + t] = ms[t];
  }
}

__global__ void k_mark_list(int32_t m, const int32_t* __restrict__ list, int32_t* __restrict__ pos) {
  const int64_t q = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (q < m) pos[list[q]] = (int32_t)q;
}

// Step 0 of the search from J = P(A~(:, k)), solved for every column by the
// register-resident float64 solver (residual norms r): a column whose residual
// is within delta keeps J (written to pad at poff[k], |J| to cntJ[k]); the
// others are flagged in todo for the search kernel, which starts them over.
__global__ void __launch_bounds__(SNT) k_spai_first(int32_t n, const int64_t* __restrict__ jptr,
                                                    const int32_t* __restrict__ jidx,
                                                    const double* __restrict__ r, double delta,
                                                    const int64_t* __restrict__ poff,
                                                    int32_t* __restrict__ pad, int32_t* __restrict__ cntJ,
                                                    int32_t* __restrict__ todo) {
  const int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (k >= n) return;
  const int64_t a = jptr[k];
  const int nJ = (int)(jptr[k + 1] - a);
  if (!(r[k] <= delta) || nJ > SJMAX) {
    todo[k] = 1;
    return;
  }
  todo[k] = 0;
  const int64_t o = poff[k];
  for (int c = 0; c < nJ; ++c) pad[o + c] = jidx[a + c];
  cntJ[k] = nJ;
}

__global__ void k_spai_ub(int32_t n, const int32_t* cp, int init, int extra, int32_t* ub) {
  const int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (k < n) ub[k] = (init == SAI_INIT_DIAG ? 1 : cp[k + 1] - cp[k]) + extra;
}

__global__ void k_compact_lists(int32_t n, const int64_t* __restrict__ poff,
                                const int32_t* __restrict__ pad, const int64_t* __restrict__ off,
                                int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * SNT + threadIdx.x;
  if (k >= n) return;
  const int64_t a = off[k], b = off[k + 1], p = poff[k];
  for (int64_t t = 0; t < b - a; ++t) out[a + t] = pad[p + t];
}

}  // namespace

void spai_patterns(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st,
                   const Allocator& al, DBuf<int64_t>& jptr, DBuf<int32_t>& jidx,
                   DBuf<int64_t>& iptr, DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ,
                   DBuf<int32_t>& cntI, int* l_m) {
  const int32_t n = sp->n;
  if (o.spai_steps < 0 || o.spai_per_step < 1 || o.spai_per_step > 16)
    SAI_THROW(SAI_EINVAL, "spai_steps >= 0 and 1 <= spai_per_step <= 16 required");
  if (o.spai_init != SAI_INIT_PATTERN_A && o.spai_init != SAI_INIT_DIAG)
    SAI_THROW(SAI_EINVAL, "bad spai_init");
  SAI_PROF("spai_search", st);
  DBuf<double> cn2(&al, (size_t)n);
  hipLaunchKernelGGL(k_colnorm2, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, sp->t_col_ptr.p,
                     sp->t_cval.p, cn2.p);
  LAUNCH_CHECK();
  DBuf<int32_t> ub(&al, (size_t)n + 1);
  hipLaunchKernelGGL(k_spai_ub, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, sp->t_col_ptr.p,
                     o.spai_init, o.spai_steps * o.spai_per_step, ub.p);
  LAUNCH_CHECK();
  DBuf<int64_t> poff(&al, (size_t)n + 1);
  exclusive_scan_i32_to_i64(ub.p, poff.p, n, al, st);
  const int64_t ptot = read_scalar(poff.p + n, st);
  DBuf<int32_t> pad(&al, (size_t)ptot + 1);
  cntJ.alloc(&al, (size_t)n + 1);
  // augmentation steps taken per column (0 for the columns that stop at step 0)
  DBuf<int32_t> taken(&al, (size_t)n + 1);
  HIPC(hipMemsetAsync(taken.p, 0, sizeof(int32_t) * ((size_t)n + 1), st));
  // From J = P(A~(:, k)), step 0 of every column runs on the static pattern
  // builder and the register-resident float64 solver; only the columns whose
  // residual exceeds delta go to the search kernel (on the irregular 200,000
  // matrix most columns stop at step 0, and one workgroup per column spent
  // 30 ms on their first solves).
  DBuf<int32_t> list;
  int nwork = n;
  if (o.spai_init == SAI_INIT_PATTERN_A && o.spai_steps > 0) {
    DBuf<int64_t> jA, iA;
    DBuf<int32_t> jiA, iiA, cJA, cIA;
    build_patterns(sp, SAI_PAT_A, st, al, jA, jiA, iA, iiA, cJA, cIA);
    DBuf<int> mx(&al, 2);
    HIPC(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_max2, dim3(grid_for(n, SNT, 256)), dim3(SNT), 0, st, n, cIA.p, cJA.p, mx.p);
    LAUNCH_CHECK();
    int hm[2];
    HIPC(hipMemcpyAsync(hm, mx.p, sizeof(hm), hipMemcpyDeviceToHost, st));
    const int64_t tot = read_scalar(jA.p + n, st);
    DBuf<double> m1(&al, (size_t)tot + 1), r1(&al, (size_t)n + 1);
    const int nsing = solve_columns<double>(sp, jA.p, jiA.p, iA.p, iiA.p, cJA.p, cIA.p, hm[0], hm[1],
                                            m1.p, r1.p, nullptr, al, st);
    if (nsing > 0)
      SAI_THROW(SAI_ESINGULAR, "%d column least-squares blocks are rank deficient", nsing);
    DBuf<int32_t> todo(&al, (size_t)n + 1);
    hipLaunchKernelGGL(k_spai_first, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, jA.p, jiA.p, r1.p,
                       o.delta, poff.p, pad.p, cntJ.p, todo.p);
    LAUNCH_CHECK();
    list.alloc(&al, (size_t)n + 1);
    DBuf<int> cnt(&al, 1);
    HIPC(hipMemsetAsync(cnt.p, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_list_flagged, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, todo.p, list.p, n,
                       cnt.p);
    LAUNCH_CHECK();
    nwork = read_scalar(cnt.p, st);
    if (nwork > 1) {
      // largest |I| of step 0 first (the order does not change any column's result)
      DBuf<int32_t> key(&al, (size_t)nwork);
      hipLaunchKernelGGL(k_gather_i32, dim3(grid_for(nwork, SNT)), dim3(SNT), 0, st, nwork, list.p, cIA.p,
                         key.p);
      LAUNCH_CHECK();
      std::vector<int32_t> hl((size_t)nwork), hk((size_t)nwork), ord((size_t)nwork), sl((size_t)nwork);
      HIPC(hipMemcpyAsync(hl.data(), list.p, sizeof(int32_t) * (size_t)nwork, hipMemcpyDeviceToHost, st));
      HIPC(hipMemcpyAsync(hk.data(), key.p, sizeof(int32_t) * (size_t)nwork, hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      for (int i = 0; i < nwork; ++i) ord[(size_t)i] = i;
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return hk[(size_t)a] > hk[(size_t)b]; });
      for (int i = 0; i < nwork; ++i) sl[(size_t)i] = hl[(size_t)ord[(size_t)i]];
      HIPC(hipMemcpyAsync(list.p, sl.data(), sizeof(int32_t) * (size_t)nwork, hipMemcpyHostToDevice, st));
      HIPC(hipStreamSynchronize(st));
    }
  }
  if (nwork > 0) {
    // one workspace slot per resident workgroup (the search is latency-bound:
    // every workgroup the device can hold at once gets a column)
    // workgroup size: eight wavefronts per column (irregular 200,000 matrix:
    // 22.5 ms with 8, 26.3 with 4, 28.2 with 16, 47.9 with 1)
    const int want = (int)tune_get("SPAI_NT", 512);
    const int bnt = (want == 64 || want == 256 || want == 1024) ? want : 512;
    DBuf<int32_t> ovf(&al, (size_t)nwork + 1);
    DBuf<int> err(&al, 3);  // error flags, work counter, overflow count
    HIPC(hipMemsetAsync(err.p, 0, 3 * sizeof(int), st));
    // runs the search over `cnt` columns of `lst` with the limits C, nslot slots
    auto search = [&](auto capc, const int32_t* lst, int cnt, int32_t* ovf_out, int* ovf_cnt, int nslot_max) {
      using C = decltype(capc);
      const void* kern = bnt == 64    ? (const void*)k_spai<64, C>
                         : bnt == 512 ? (const void*)k_spai<512, C>
                         : bnt == 1024 ? (const void*)k_spai<1024, C>
                                       : (const void*)k_spai<256, C>;
      const int nslot = (int)std::min<int64_t>(
          {(int64_t)cnt, (int64_t)nslot_max, (int64_t)tune_get("SPAI_SLOTS", resident_blocks(kern, bnt))});
      DBuf<int32_t> wI(&al, (size_t)nslot * C::I), wc(&al, (size_t)nslot * C::N),
          wo(&al, (size_t)nslot * (C::I + 1)), wS(&al, (size_t)nslot * C::I), wP(&al, (size_t)nslot * C::I);
      DBuf<double> wW(&al, (size_t)nslot * C::I * (C::J + 1)), wr(&al, (size_t)nslot * C::I),
          wg(&al, (size_t)nslot * C::N);
      HIPC(hipMemsetAsync(err.p + 1, 0, sizeof(int), st));
      Ws ws{wI.p, wc.p, wo.p, wW.p, wr.p, wg.p, wS.p, wP.p};
      auto go = [&](auto k) {
        hipLaunchKernelGGL(k, dim3(nslot), dim3(bnt), 0, st, n, sp->t_col_ptr.p, sp->t_row_idx.p,
                           sp->t_cval.p, sp->t_row_ptr.p, sp->t_col_idx.p, cn2.p, o.spai_steps,
                           o.spai_per_step, o.delta, o.spai_init, poff.p, pad.p, cntJ.p, ws, lst,
                           (int32_t)cnt, err.p + 1, err.p, taken.p, ovf_out, ovf_cnt);
      };
      if (bnt == 64) go(k_spai<64, C>);
      else if (bnt == 512) go(k_spai<512, C>);
      else if (bnt == 1024) go(k_spai<1024, C>);
      else go(k_spai<256, C>);
      LAUNCH_CHECK();
      HIPC(hipStreamSynchronize(st));  // the workspaces are released on return
    };
    search(CapS{}, (const int32_t*)list.p, nwork, ovf.p, err.p + 2, NSLOT_MAX);
    int hs[3];
    HIPC(hipMemcpyAsync(hs, err.p, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (hs[0] & E_SING)
      SAI_THROW(SAI_ESINGULAR, "a column least-squares block of the SPAI search is rank deficient");
    if (hs[2] > 0) {
      // columns that outgrew the small limits, searched again from their start
      search(CapL{}, (const int32_t*)ovf.p, hs[2], nullptr, nullptr, NSLOT_L);
      HIPC(hipMemcpyAsync(hs, err.p, sizeof(hs), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      if (hs[0] & E_SING)
        SAI_THROW(SAI_ESINGULAR, "a column least-squares block of the SPAI search is rank deficient");
    }
    if (hs[0] & E_TOOBIG)
      SAI_THROW(SAI_ETOOBIG, "SPAI search exceeded |J| <= %d, |I| <= %d or %d candidates", CapL::J, CapL::I,
                CapL::N);
  }
  if (l_m) {
    DBuf<int> mx(&al, 2);
    HIPC(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_max2, dim3(grid_for(n, SNT, 256)), dim3(SNT), 0, st, n, taken.p, taken.p, mx.p);
    LAUNCH_CHECK();
    *l_m = read_scalar(mx.p, st);
  }
  jptr.alloc(&al, (size_t)n + 1);
  exclusive_scan_i32_to_i64(cntJ.p, jptr.p, n, al, st);
  const int64_t jtot = read_scalar(jptr.p + n, st);
  jidx.alloc(&al, (size_t)jtot + 1);
  hipLaunchKernelGGL(k_compact_lists, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, poff.p, pad.p,
                     jptr.p, jidx.p);
  LAUNCH_CHECK();
  rows_of_patterns(sp, st, al, jptr, jidx, iptr, iidx, cntI);
}

// PSAI(tol): final patterns J_k (packed), their values (float64, packed), the
// residual norms of the last solves, and |J_k|; I_k for the statistics and
// inspection.
void psai_patterns(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st,
                   const Allocator& al, DBuf<int64_t>& jptr, DBuf<int32_t>& jidx,
                   DBuf<int64_t>& iptr, DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ,
                   DBuf<int32_t>& cntI, DBuf<double>& mval, DBuf<double>& res, int* l_m) {
  const int32_t n = sp->n;
  if (o.psai_lmax < 0 || o.psai_lmax > 64) SAI_THROW(SAI_EINVAL, "psai_lmax must be in [0, 64]");
  if (!(o.delta > 0.0)) SAI_THROW(SAI_EINVAL, "delta must be > 0");
  SAI_PROF("psai_search", st);
  // ||A~||_1
  double a1 = 0.0;
  {
    DBuf<double> cs(&al, (size_t)n);
    hipLaunchKernelGGL(k_colabs, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, sp->t_col_ptr.p,
                       sp->t_cval.p, cs.p);
    LAUNCH_CHECK();
    std::vector<double> h((size_t)n);
    HIPC(hipMemcpyAsync(h.data(), cs.p, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    for (double v : h) a1 = std::max(a1, v);
  }
  if (!(a1 > 0.0)) SAI_THROW(SAI_EINVAL, "A~ is zero");
  DBuf<int32_t> jpad(&al, (size_t)n * SJMAX);
  DBuf<double> mpad(&al, (size_t)n * SJMAX);
  cntJ.alloc(&al, (size_t)n + 1);
  res.alloc(&al, (size_t)n + 1);
  DBuf<int32_t> todo(&al, (size_t)n + 1);
  DBuf<int32_t> loops(&al, (size_t)n + 1);  // loops run per column
  // ---- loop l = 0 on J_k = P(A~(:, k)) with the register-resident column solver
  {
    DBuf<int64_t> jA, iA;
    DBuf<int32_t> jiA, iiA, cJA, cIA;
    build_patterns(sp, SAI_PAT_A, st, al, jA, jiA, iA, iiA, cJA, cIA);
    DBuf<int> mx(&al, 2);
    HIPC(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_max2, dim3(grid_for(n, SNT, 256)), dim3(SNT), 0, st, n, cIA.p, cJA.p, mx.p);
    LAUNCH_CHECK();
    int hm[2];
    HIPC(hipMemcpyAsync(hm, mx.p, sizeof(hm), hipMemcpyDeviceToHost, st));
    const int64_t tot = read_scalar(jA.p + n, st);
    DBuf<double> m1(&al, (size_t)tot + 1), r1(&al, (size_t)n + 1);
    const int nsing = solve_columns<double>(sp, jA.p, jiA.p, iA.p, iiA.p, cJA.p, cIA.p, hm[0], hm[1],
                                            m1.p, r1.p, nullptr, al, st);
    if (nsing > 0)
      SAI_THROW(SAI_ESINGULAR, "%d column least-squares blocks are rank deficient", nsing);
    hipLaunchKernelGGL(k_psai_first, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, jA.p, jiA.p, m1.p,
                       r1.p, o.delta, a1, o.psai_lmax, jpad.p, mpad.p, cntJ.p, res.p, todo.p, loops.p);
    LAUNCH_CHECK();
  }
  // ---- the other columns: the whole loop in the search kernel
  DBuf<int32_t> list(&al, (size_t)n + 1);
  DBuf<int> cnt(&al, 1);
  HIPC(hipMemsetAsync(cnt.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_list_flagged, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, todo.p, list.p, n,
                     cnt.p);
  LAUNCH_CHECK();
  const int ntodo = read_scalar(cnt.p, st);
  // columns that outgrow the small limits: searched again with the large ones,
  // their results in rows of bigJ / bigM (bigpos[k] = row, else -1)
  DBuf<int32_t> bigJ, bigpos;
  DBuf<double> bigM;
  int nbig = 0;
  if (ntodo > 0) {
    // one wavefront per column: the problems of the first loops are small, and
    // more columns in flight pay more than threads per column (100^3 matrix,
    // every column through this kernel: 52 -> 34 ms); the SPAI search, with
    // larger problems, keeps four
    const int bnt = tune_get("PSAI_NT", 64) == 256 ? 256 : 64;
    DBuf<int32_t> ovf(&al, (size_t)ntodo + 1);
    DBuf<int> err(&al, 2);  // error flags, overflow count
    HIPC(hipMemsetAsync(err.p, 0, 2 * sizeof(int), st));
    auto search = [&](auto capc, int bthreads, const int32_t* lst, int m, int32_t* jout, double* mout,
                      int out_list, int32_t* ovf_out, int* ovf_cnt, int nslot_max) {
      using C = decltype(capc);
      const void* kern = bthreads == 64 ? (const void*)k_psai<64, C> : (const void*)k_psai<256, C>;
      const int nslot = (int)std::min<int64_t>(
          {(int64_t)m, (int64_t)nslot_max, (int64_t)tune_get("SPAI_SLOTS", resident_blocks(kern, bthreads))});
      DBuf<int32_t> wI(&al, (size_t)nslot * C::I), wc(&al, (size_t)nslot * C::N),
          wo(&al, (size_t)nslot * (C::I + 1)), wf(&al, (size_t)nslot * C::I);
      DBuf<double> wW(&al, (size_t)nslot * C::I * (C::J + 1)), wr(&al, (size_t)nslot * C::I),
          wg(&al, (size_t)nslot * C::N);
      Ws ws{wI.p, wc.p, wo.p, wW.p, wr.p, wg.p};
      auto go = [&](auto k) {
        hipLaunchKernelGGL(k, dim3(nslot), dim3(bthreads), 0, st, n, sp->t_col_ptr.p, sp->t_row_idx.p,
                           sp->t_cval.p, o.psai_lmax, o.delta, a1, jout, mout, cntJ.p, res.p, ws, wf.p, lst,
                           (int32_t)m, err.p, loops.p, out_list, ovf_out, ovf_cnt);
      };
      if (bthreads == 64) go(k_psai<64, C>);
      else go(k_psai<256, C>);
      LAUNCH_CHECK();
      HIPC(hipStreamSynchronize(st));  // the workspaces are released on return
    };
    search(CapS{}, bnt, (const int32_t*)list.p, ntodo, jpad.p, mpad.p, 0, ovf.p, err.p + 1, NSLOT_MAX);
    int hs[2];
    HIPC(hipMemcpyAsync(hs, err.p, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    nbig = hs[1];
    if (!(hs[0] & E_SING) && nbig > 0) {
      bigJ.alloc(&al, (size_t)nbig * CapL::J);
      bigM.alloc(&al, (size_t)nbig * CapL::J);
      bigpos.alloc(&al, (size_t)n + 1);
      fill_i32(bigpos.p, -1, n, st);
      hipLaunchKernelGGL(k_mark_list, dim3(grid_for(nbig, SNT)), dim3(SNT), 0, st, nbig,
                         (const int32_t*)ovf.p, bigpos.p);
      LAUNCH_CHECK();
      // larger problems: four wavefronts per column
      search(CapL{}, 256, (const int32_t*)ovf.p, nbig, bigJ.p, bigM.p, 1, nullptr, nullptr, NSLOT_L);
      HIPC(hipMemcpyAsync(hs, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
    }
    if (hs[0] & E_SING)
      SAI_THROW(SAI_ESINGULAR, "a column least-squares block of the PSAI(tol) loop is rank deficient");
    if (hs[0] & E_TOOBIG)
      SAI_THROW(SAI_ETOOBIG, "PSAI(tol) exceeded |J| <= %d, |I| <= %d or %d gathered entries", CapL::J,
                CapL::I, CapL::N);
  }
  if (l_m) {
    DBuf<int> mx(&al, 2);
    HIPC(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_max2, dim3(grid_for(n, SNT, 256)), dim3(SNT), 0, st, n, loops.p, loops.p, mx.p);
    LAUNCH_CHECK();
    *l_m = read_scalar(mx.p, st);
  }
  jptr.alloc(&al, (size_t)n + 1);
  exclusive_scan_i32_to_i64(cntJ.p, jptr.p, n, al, st);
  const int64_t jtot = read_scalar(jptr.p + n, st);
  jidx.alloc(&al, (size_t)jtot + 1);
  mval.alloc(&al, (size_t)jtot + 1);
  hipLaunchKernelGGL(k_compact_psai, dim3(grid_for(n, SNT)), dim3(SNT), 0, st, n, jpad.p, mpad.p,
                     jptr.p, jidx.p, mval.p, (const int32_t*)bigpos.p, (const int32_t*)bigJ.p,
                     (const double*)bigM.p);
  LAUNCH_CHECK();
  rows_of_patterns(sp, st, al, jptr, jidx, iptr, iidx, cntI);
}

}  // namespace sai
