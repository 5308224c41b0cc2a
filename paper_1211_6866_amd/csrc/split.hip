// Split A = A~ + U V^T on the device (Procedure * step 1; Section 3 (split);
// Section 4, first and second issues).
//
// p = floor(nnz/n); irregular columns are those with more than factor*p
// nonzeros; each keeps its diagonal plus keep-1 off-diagonal entries chosen by
// the smallest key (|i-j|, i) ("nearest", the paper's choice) or (-|a_ij|, i)
// ("largest"); the rest move to U.  Every step is integer/index work or a value
// copy, so the result is exact.
#include "sai_internal.hpp"

namespace sai {
namespace {

constexpr int NT = 256;

enum { ERR_PTR = 1, ERR_COL = 2, ERR_ORDER = 4, ERR_VAL = 8, ERR_ZERODIAG = 16 };

// Wave-cooperative traversal of a CSR block: the wavefront owns rows r0 ..
// r0+63 and walks their entries (contiguous in memory) 64 at a time, so that
// the reads of the entries are coalesced; the row of entry e is found by a
// binary search over the 64 row starts held one per lane.
struct WaveRows {
  int64_t r0;
  int32_t myrp;  // start of row r0 + lane (the end of the block for lanes past n)
  int32_t e0, e1;
  __device__ WaveRows(int32_t n, const int32_t* __restrict__ rp, int64_t r0_) : r0(r0_) {
    const int lane = threadIdx.x & 63;
    const int64_t r = r0 + lane;
    const int64_t rend = min<int64_t>(r0 + 64, n);
    myrp = rp[min<int64_t>(r, rend)];
    e0 = __shfl(myrp, 0, 64);
    e1 = rp[rend];
  }
  // tile-relative row (0..63) of entry e, e0 <= e < e1; every lane must call it
  __device__ int row_of(int32_t e) const {
    int lo = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const int cand = lo + step;
      const int32_t v = __shfl(myrp, cand & 63, 64);
      if (cand < 64 && v <= e) lo = cand;
    }
    return lo;
  }
};

// wavefronts of a 256-thread block, one 64-row block of rows each (grid-stride)
#define WAVE_ROW_BLOCKS(n)                                                                   \
  for (int64_t r0_ = ((int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * 64; r0_ < (n); \
       r0_ += (int64_t)gridDim.x * NT)


// Column counts are kept in CSTRIPE stripes (stripe = row mod CSTRIPE, layout
// [stripe][n]), so that the many entries of an irregular column do not all
// queue on one counter; k_dense_flag adds the stripes.
constexpr int CSTRIPE = 8;

// Checks the CSR input (row pointers monotone within [0, nnz], column indices
// in range and strictly increasing within a row, finite values) and counts
// the entries of every column.  A block of 64 rows whose row pointers are bad
// is flagged and not read further.
__global__ void __launch_bounds__(NT) k_validate_count(int32_t n, int64_t nnz,
                                                       const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val,
                                                       int32_t* __restrict__ colcnt8, int* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz))
    atomicOr(err, ERR_PTR);
  WAVE_ROW_BLOCKS(n) {
    const int64_t r = r0_ + lane;
    bool bad = false;
    if (r < n) {
      const int32_t a = row_ptr[r], b = row_ptr[r + 1];
      bad = b < a || a < 0 || (int64_t)b > nnz;
    }
    if (__any(bad)) {
      if (lane == 0) atomicOr(err, ERR_PTR);
      continue;
    }
    const WaveRows w(n, row_ptr, r0_);
    int e_local = 0;
    for (int32_t base = w.e0; base < w.e1; base += 64) {
      const int32_t e = base + lane;
      const int t = w.row_of(min(e, w.e1 - 1));
      const int32_t rs = __shfl(w.myrp, t, 64);
      if (e < w.e1) {
        const int32_t j = col[e];
        if (j < 0 || j >= n) {
          e_local |= ERR_COL;
        } else {
          if (e > rs && col[e - 1] >= j) e_local |= ERR_ORDER;
          if (!isfinite(val[e])) e_local |= ERR_VAL;
          atomicAdd(&colcnt8[(int64_t)(t % CSTRIPE) * n + j], 1);
        }
      }
    }
    if (__any(e_local != 0) && e_local) atomicOr(err, e_local);
  }
}

__global__ void k_dense_flag(int32_t n, const int32_t* __restrict__ colcnt8, double thr,
                             int32_t* __restrict__ colcnt, int32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  int32_t c = 0;
#pragma unroll
  for (int q = 0; q < CSTRIPE; ++q) c += colcnt8[(int64_t)q * n + j];
  colcnt[j] = c;
  flag[j] = ((double)c > thr) ? 1 : 0;
}

// The irregular columns given by the caller (flag cleared beforehand).
__global__ void k_flag_set(int32_t s, const int32_t* __restrict__ list, int32_t* __restrict__ flag) {
  const int64_t d = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (d < s) flag[list[d]] = 1;
}

__global__ void k_dense_compact(int32_t n, const int32_t* flag, const int32_t* pos,
                                const int32_t* colcnt, int32_t* dense_cols, int32_t* dcount,
                                int32_t* colmap) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  if (flag[j]) {
    const int32_t d = pos[j];
    dense_cols[d] = (int32_t)j;
    dcount[d] = colcnt[j];
    colmap[j] = d;
  } else {
    colmap[j] = -1;
  }
}

// Collect (row, CSR position) of every entry of every irregular column.
__global__ void k_dense_gather(int32_t n, const int32_t* __restrict__ row_ptr,
                               const int32_t* __restrict__ col, const int32_t* __restrict__ colmap,
                               const int64_t* __restrict__ doff, int32_t* __restrict__ dcur,
                               int32_t* __restrict__ lrow, int32_t* __restrict__ lpos) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int32_t a = i < n ? row_ptr[i] : 0;
  const int32_t len = i < n ? row_ptr[i + 1] - a : 0;
  int mx = len;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, WAVE));
  // wave-uniform trip count so that the aggregated atomics see every lane
  for (int32_t t = 0; t < mx; ++t) {
    const int32_t e = a + t;
    const int32_t d = t < len ? colmap[col[e]] : -1;
    const int32_t slot = agg_slot(dcur, d);
    if (d >= 0) {
      lrow[doff[d] + slot] = (int32_t)i;
      lpos[doff[d] + slot] = e;
    }
  }
}

// Contention-free variant of the gather for s <= GATHER_SMAX: each block counts
// the irregular-column entries of its rows in LDS (pass 0), a prefix sum over the
// (column, block) counts in column-major order gives every block its slice of
// every column's list, and pass 1 scatters into those slices.
constexpr int GATHER_ROWS = 4096;
constexpr int GATHER_SMAX = 1024;

__global__ void __launch_bounds__(NT) k_dense_gather_blk(int32_t n, int s, const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ colmap, int pass,
                                                         int32_t* __restrict__ bcnt,
                                                         const int64_t* __restrict__ boff,
                                                         int32_t* __restrict__ lrow,
                                                         int32_t* __restrict__ lpos) {
  __shared__ int32_t cnt[GATHER_SMAX];
  const int nb = gridDim.x;
  for (int d = threadIdx.x; d < s; d += NT) cnt[d] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * GATHER_ROWS;
  const int64_t r1 = min<int64_t>(n, r0 + GATHER_ROWS);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int32_t d = colmap[col[e]];
      if (d < 0) continue;
      const int32_t slot = atomicAdd(&cnt[d], 1);
      if (pass == 1) {
        const int64_t o = boff[(int64_t)d * nb + blockIdx.x] + slot;
        lrow[o] = (int32_t)i;
        lpos[o] = e;
      }
    }
  }
  __syncthreads();
  if (pass == 0)
    for (int d = threadIdx.x; d < s; d += NT) bcnt[(int64_t)d * nb + blockIdx.x] = cnt[d];
}

struct Key {
  double a;
  int32_t i;
};
__device__ __forceinline__ bool key_less(const Key& x, const Key& y) {
  return x.a < y.a || (x.a == y.a && x.i < y.i);
}

// One workgroup per irregular column: choose the keep-1 smallest keys among the
// off-diagonal entries by keep-1 rounds of "smallest key above the previous
// one"; mark the others as dropped.
__global__ void __launch_bounds__(NT) k_dense_select(const int32_t* __restrict__ dense_cols,
                                                     const int64_t* __restrict__ doff,
                                                     const int32_t* __restrict__ dcount,
                                                     const int32_t* __restrict__ lrow,
                                                     const int32_t* __restrict__ lpos,
                                                     const double* __restrict__ val, int keep,
                                                     int rule, uint8_t* __restrict__ drop,
                                                     int* __restrict__ err) {
  __shared__ double sa[NT];
  __shared__ int32_t si[NT];
  __shared__ int has_diag;
  const int d = blockIdx.x;
  const int32_t j = dense_cols[d];
  const int64_t off = doff[d];
  const int32_t cnt = dcount[d];
  if (threadIdx.x == 0) has_diag = 0;
  __syncthreads();
  for (int32_t t = threadIdx.x; t < cnt; t += NT)
    if (lrow[off + t] == j) has_diag = 1;
  __syncthreads();
  if (!has_diag) {
    if (threadIdx.x == 0) atomicOr(err, ERR_ZERODIAG);
    return;
  }
  Key last{-INFINITY, -1};
  bool have = false;  // at least one key selected
  for (int r = 0; r < keep - 1; ++r) {
    Key best{INFINITY, 0x7fffffff};
    for (int32_t t = threadIdx.x; t < cnt; t += NT) {
      const int32_t i = lrow[off + t];
      if (i == j) continue;
      Key k;
      k.i = i;
      k.a = (rule == SAI_KEEP_NEAREST) ? (double)(i > j ? i - j : j - i) : -fabs(val[lpos[off + t]]);
      if (key_less(last, k) && key_less(k, best)) best = k;
    }
    sa[threadIdx.x] = best.a;
    si[threadIdx.x] = best.i;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        Key x{sa[threadIdx.x], si[threadIdx.x]}, y{sa[threadIdx.x + o], si[threadIdx.x + o]};
        if (key_less(y, x)) { sa[threadIdx.x] = y.a; si[threadIdx.x] = y.i; }
      }
      __syncthreads();
    }
    Key b{sa[0], si[0]};
    __syncthreads();
    if (b.i == 0x7fffffff) break;  // fewer off-diagonals than keep-1
    last = b;
    have = true;
  }
  for (int32_t t = threadIdx.x; t < cnt; t += NT) {
    const int32_t i = lrow[off + t];
    if (i == j) continue;
    bool kept = false;
    if (have) {
      Key k;
      k.i = i;
      k.a = (rule == SAI_KEEP_NEAREST) ? (double)(i > j ? i - j : j - i) : -fabs(val[lpos[off + t]]);
      kept = !key_less(last, k);  // k <= last
    }
    if (!kept) drop[lpos[off + t]] = 1;
  }
}

// Same selection in one pass over the column for keep - 1 <= SEL_K: every
// thread keeps the keep - 1 smallest keys of its entries, sorted, in registers;
// then keep - 1 rounds of a block minimum over the threads' current heads (the
// thread whose head is taken moves to its next key) yield the keep - 1
// smallest keys of the column (keys are distinct: one per row).
constexpr int SEL_K = 16;

template <int B = NT>
__device__ __forceinline__ Key block_min_key(Key k, double* sa, int32_t* si) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Key y{__shfl_xor(k.a, o, 64), __shfl_xor(k.i, o, 64)};
    if (key_less(y, k)) k = y;
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = k.a;
    si[w] = k.i;
  }
  __syncthreads();
  Key b{sa[0], si[0]};
#pragma unroll
  for (int q = 1; q < B / 64; ++q) {
    Key y{sa[q], si[q]};
    if (key_less(y, b)) b = y;
  }
  __syncthreads();
  return b;
}

// one 1024-thread workgroup per irregular column: each scans ~1/1024 of its entries
constexpr int SEL_NT = 1024;
__global__ void __launch_bounds__(SEL_NT) k_dense_select_k(const int32_t* __restrict__ dense_cols,
                                                       const int64_t* __restrict__ doff,
                                                       const int32_t* __restrict__ dcount,
                                                       const int32_t* __restrict__ lrow,
                                                       const int32_t* __restrict__ lpos,
                                                       const double* __restrict__ val, int keep,
                                                       int rule, uint8_t* __restrict__ drop,
                                                       int* __restrict__ err) {
  __shared__ double sa[SEL_NT / 64];
  __shared__ int32_t si[SEL_NT / 64];
  __shared__ int has_diag;
  const int d = blockIdx.x;
  const int32_t j = dense_cols[d];
  const int64_t off = doff[d];
  const int32_t cnt = dcount[d];
  const int K = keep - 1;  // <= SEL_K (checked by the caller)
  if (threadIdx.x == 0) has_diag = 0;
  __syncthreads();
  double ka[SEL_K];
  int32_t ki[SEL_K];
#pragma unroll
  for (int u = 0; u < SEL_K; ++u) {
    ka[u] = INFINITY;
    ki[u] = 0x7fffffff;
  }
  bool diag = false;
  for (int32_t t = threadIdx.x; t < cnt; t += SEL_NT) {
    const int32_t i = lrow[off + t];
    if (i == j) {
      diag = true;
      continue;
    }
    Key k;
    k.i = i;
    k.a = (rule == SAI_KEEP_NEAREST) ? (double)(i > j ? i - j : j - i) : -fabs(val[lpos[off + t]]);
    // insert into the sorted list of the K smallest (slots >= K stay empty)
#pragma unroll
    for (int u = SEL_K - 1; u >= 0; --u) {
      if (u < K) {
        const Key cur{ka[u], ki[u]};
        const Key prev = u > 0 ? Key{ka[u - 1], ki[u - 1]} : Key{-INFINITY, -1};
        if (key_less(k, cur)) {
          if (key_less(k, prev)) {
            ka[u] = prev.a;  // shift up
            ki[u] = prev.i;
          } else {
            ka[u] = k.a;  // k goes here
            ki[u] = k.i;
          }
        }
      }
    }
  }
  if (diag) has_diag = 1;
  __syncthreads();
  if (!has_diag) {
    if (threadIdx.x == 0) atomicOr(err, ERR_ZERODIAG);
    return;
  }
  Key last{-INFINITY, -1};
  bool have = false;
  int head = 0;
  for (int r = 0; r < K; ++r) {
    Key mine{INFINITY, 0x7fffffff};
#pragma unroll
    for (int u = 0; u < SEL_K; ++u)
      if (u == head) mine = Key{ka[u], ki[u]};
    const Key b = block_min_key<SEL_NT>(mine, sa, si);
    if (b.i == 0x7fffffff) break;  // fewer off-diagonals than keep-1
    if (b.i == mine.i && head < SEL_K) ++head;
    last = b;
    have = true;
  }
  for (int32_t t = threadIdx.x; t < cnt; t += SEL_NT) {
    const int32_t i = lrow[off + t];
    if (i == j) continue;
    bool kept = false;
    if (have) {
      Key k;
      k.i = i;
      k.a = (rule == SAI_KEEP_NEAREST) ? (double)(i > j ? i - j : j - i) : -fabs(val[lpos[off + t]]);
      kept = !key_less(last, k);  // k <= last
    }
    if (!kept) drop[lpos[off + t]] = 1;
  }
}

__global__ void k_row_counts(int32_t n, const int32_t* __restrict__ row_ptr,
                             const uint8_t* __restrict__ drop, int32_t* __restrict__ tcnt,
                             int32_t* __restrict__ ucnt) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  int32_t t = 0, u = 0;
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    if (drop[e]) ++u; else ++t;
  }
  tcnt[i] = t;
  ucnt[i] = u;
}

__global__ void k_row_scatter(int32_t n, const int32_t* __restrict__ row_ptr,
                              const int32_t* __restrict__ col, const double* __restrict__ val,
                              const uint8_t* __restrict__ drop, const int32_t* __restrict__ colmap,
                              const int32_t* __restrict__ t_row_ptr, int32_t* __restrict__ t_col,
                              double* __restrict__ t_val, const int32_t* __restrict__ u_row_ptr,
                              int32_t* __restrict__ u_col, double* __restrict__ u_val) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  int32_t pt = t_row_ptr[i], pu = u_row_ptr[i];
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    if (drop[e]) {
      u_col[pu] = colmap[col[e]];
      u_val[pu] = val[e];
      ++pu;
    } else {
      t_col[pt] = col[e];
      t_val[pt] = val[e];
      ++pt;
    }
  }
}

}  // namespace

// ---- CSR -> CSC transpose (shared with the build) ----------------------------

// One thread per row: the entries u of consecutive rows fall in different
// columns, so the atomics of a wavefront instruction rarely collide.
__global__ void __launch_bounds__(NT) k_tr_count(int32_t n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) atomicAdd(&cnt[ci[e]], 1);
}

// One thread per row, its entries TB at a time: the TB slot reservations
// (atomics that return a value) are all in flight before the first is used.
template <class V>
__global__ void __launch_bounds__(NT) k_tr_scatter(int32_t n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const V* __restrict__ v,
                                                   const int32_t* __restrict__ cp, int32_t* __restrict__ cur,
                                                   int32_t* __restrict__ ri, V* __restrict__ cv) {
  constexpr int TB = 8;
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int32_t a = rp[i], b = rp[i + 1];
  for (int32_t e = a; e < b; e += TB) {
    int32_t j[TB], slot[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) j[u] = e + u < b ? ci[e + u] : -1;
#pragma unroll
    for (int u = 0; u < TB; ++u) slot[u] = j[u] >= 0 ? atomicAdd(&cur[j[u]], 1) : 0;
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      if (j[u] >= 0) {
        const int32_t q = cp[j[u]] + slot[u];
        ri[q] = (int32_t)i;
        cv[q] = v[e + u];
      }
    }
  }
}

// Sort the segment lo .. lo+len-1 (len <= 32) of (K, W) by key with a bitonic
// network in registers (all indices static).
template <class V, class KP, class WP>
__device__ __forceinline__ void sort_seg32(KP K, WP W, int64_t lo, int len) {
  int32_t key[32];
  V val[32];
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    key[t] = t < len ? K[lo + t] : 0x7fffffff;
    val[t] = t < len ? W[lo + t] : V(0);
  }
#pragma unroll
  for (int kk = 2; kk <= 32; kk <<= 1) {
#pragma unroll
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
#pragma unroll
      for (int t = 0; t < 32; ++t) {
        const int l = t ^ jj;
        if (l > t) {
          const bool up = (t & kk) == 0;
          const bool sw = (key[t] > key[l]) == up;
          const int32_t k0 = key[t], k1 = key[l];
          const V v0 = val[t], v1 = val[l];
          key[t] = sw ? k1 : k0;
          key[l] = sw ? k0 : k1;
          val[t] = sw ? v1 : v0;
          val[l] = sw ? v0 : v1;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    if (t < len) {
      K[lo + t] = key[t];
      W[lo + t] = val[t];
    }
  }
}

// Sort each column segment by row (segments are short for the regular sparse
// matrices this is used on).  Makes the transpose deterministic.  A block's
// segments are contiguous: when they hold at most TS_CAP entries and none is
// longer than 32, they are staged in LDS with coalesced loads and stores and
// each thread sorts its segment there; otherwise each thread sorts in global
// memory (the register network up to 32 entries, insertion sort beyond).
constexpr int TS_NT = 64, TS_CAP = 2048;
template <class V>
__global__ void __launch_bounds__(TS_NT) k_tr_sort(int32_t m, const int32_t* __restrict__ cp,
                                                   int32_t* __restrict__ ri, V* __restrict__ cv) {
  __shared__ int32_t sk[TS_CAP];
  __shared__ V sv[TS_CAP];
  const int64_t jb = (int64_t)blockIdx.x * TS_NT;
  const int64_t jl = min<int64_t>(m, jb + TS_NT);
  const int64_t j = jb + threadIdx.x;
  const int32_t eb = cp[jb], el = cp[jl];
  const int32_t a = j < m ? cp[j] : el, b = j < m ? cp[j + 1] : el;
  // one wavefront per block: the ballot is the block's
  const bool staged = el - eb <= TS_CAP && __ballot(b - a > 32) == 0;
  if (staged) {
    for (int q = threadIdx.x; q < el - eb; q += TS_NT) {
      sk[q] = ri[eb + q];
      sv[q] = cv[eb + q];
    }
    __syncthreads();
    if (j < m) sort_seg32<V>(sk, sv, (int64_t)(a - eb), b - a);
    __syncthreads();
    for (int q = threadIdx.x; q < el - eb; q += TS_NT) {
      ri[eb + q] = sk[q];
      cv[eb + q] = sv[q];
    }
    return;
  }
  if (j >= m) return;
  if (b - a <= 32) {
    sort_seg32<V>(ri, cv, (int64_t)a, b - a);
    return;
  }
  for (int32_t x = a + 1; x < b; ++x) {
    const int32_t r = ri[x];
    const V w = cv[x];
    int32_t y = x - 1;
    while (y >= a && ri[y] > r) {
      ri[y + 1] = ri[y];
      cv[y + 1] = cv[y];
      --y;
    }
    ri[y + 1] = r;
    cv[y + 1] = w;
  }
}

template <class V>
void csr_transpose(int32_t nrows, int32_t ncols, const int32_t* rp, const int32_t* ci, const V* v,
                   int32_t* cp, int32_t* ri, V* cv, const Allocator& al, hipStream_t st) {
  DBuf<int32_t> cnt(&al, (size_t)ncols + 1);
  HIPC(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * ((size_t)ncols + 1), st));
  hipLaunchKernelGGL(k_tr_count, dim3(grid_for(nrows, NT)), dim3(NT), 0, st, nrows, rp, ci, cnt.p);
  LAUNCH_CHECK();
  exclusive_scan_i32(cnt.p, cp, ncols, al, st);
  HIPC(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * ((size_t)ncols + 1), st));
  hipLaunchKernelGGL((k_tr_scatter<V>), dim3(grid_for(nrows, NT)), dim3(NT), 0, st, nrows, rp, ci, v, cp,
                     cnt.p, ri, cv);
  LAUNCH_CHECK();
  hipLaunchKernelGGL((k_tr_sort<V>), dim3(grid_for(ncols, TS_NT)), dim3(TS_NT), 0, st, ncols, cp, ri, cv);
  LAUNCH_CHECK();
}

template void csr_transpose<double>(int32_t, int32_t, const int32_t*, const int32_t*, const double*,
                                    int32_t*, int32_t*, double*, const Allocator&, hipStream_t);
template void csr_transpose<float>(int32_t, int32_t, const int32_t*, const int32_t*, const float*,
                                   int32_t*, int32_t*, float*, const Allocator&, hipStream_t);

void split_impl(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                const double* val, const sai_split_opts& o, const Allocator& al_in, sai_split_s* h) {
  // every buffer (temporary or owned by the handle) refers to the handle's allocator,
  // which lives as long as the handle
  h->al = al_in;
  const Allocator& al = h->al;
  hipStream_t st = al.stream;
  SAI_PROF("split", st);
  if (n <= 0 || nnz < 0 || nnz >= (int64_t)INT32_MAX || !row_ptr || (nnz > 0 && (!col_idx || !val)))
    SAI_THROW(SAI_EINVAL, "bad CSR arguments (n=%d nnz=%lld)", n, (long long)nnz);
  if (!(o.dense_factor > 0.0)) SAI_THROW(SAI_EINVAL, "dense_factor must be > 0");
  if (o.rule != SAI_KEEP_NEAREST && o.rule != SAI_KEEP_LARGEST) SAI_THROW(SAI_EINVAL, "bad rule");
  const bool given = o.host_dense_cols != nullptr;
  if (given) {
    if (o.s_given < 0 || o.s_given > n) SAI_THROW(SAI_EINVAL, "s_given must be in [0, n]");
    for (int32_t d = 0; d < o.s_given; ++d) {
      const int32_t j = o.host_dense_cols[d];
      if (j < 0 || j >= n || (d > 0 && j <= o.host_dense_cols[d - 1]))
        SAI_THROW(SAI_EINVAL, "host_dense_cols must be strictly ascending in [0, n)");
    }
  }
  h->n = n;
  h->nnz_a = nnz;
  const int32_t p = (int32_t)(nnz / n);
  h->p = p;
  const int32_t keep = o.keep > 0 ? o.keep : (p > 0 ? p : 1);
  h->keep = keep;

  DBuf<int32_t> colcnt(&al, (size_t)n + 1), flag(&al, (size_t)n + 1), pos(&al, (size_t)n + 1),
      colmap(&al, (size_t)n);
  DBuf<int> err(&al, 4);
  {
    DBuf<int32_t> colcnt8(&al, (size_t)CSTRIPE * n);
    HIPC(hipMemsetAsync(colcnt8.p, 0, sizeof(int32_t) * (size_t)CSTRIPE * n, st));
    HIPC(hipMemsetAsync(err.p, 0, sizeof(int) * 4, st));
    hipLaunchKernelGGL(k_validate_count, dim3(grid_for(((int64_t)n + 63) / 64 * 64, NT, 4096)), dim3(NT), 0, st, n,
                       nnz, row_ptr, col_idx, val, colcnt8.p, err.p);
    LAUNCH_CHECK();
    const double thr = o.dense_factor * (double)p;
    hipLaunchKernelGGL(k_dense_flag, dim3(grid_for(n, NT)), dim3(NT), 0, st, n, colcnt8.p, thr, colcnt.p,
                       flag.p);
  }
  LAUNCH_CHECK();
  if (given) {
    // the caller's list replaces the count rule
    HIPC(hipMemsetAsync(flag.p, 0, sizeof(int32_t) * (size_t)n, st));
    if (o.s_given > 0) {
      DBuf<int32_t> dl(&al, (size_t)o.s_given);
      HIPC(hipMemcpyAsync(dl.p, o.host_dense_cols, sizeof(int32_t) * (size_t)o.s_given,
                          hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_flag_set, dim3(grid_for(o.s_given, NT)), dim3(NT), 0, st, o.s_given, dl.p,
                         flag.p);
      LAUNCH_CHECK();
      HIPC(hipStreamSynchronize(st));
    }
  }
  exclusive_scan_i32(flag.p, pos.p, n, al, st);
  HostStage hs(64);
  HIPC(hipMemcpyAsync(hs.as<int32_t>(), pos.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(hs.as<int32_t>() + 1, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  const int32_t s = hs.as<int32_t>()[0];
  const int e0 = hs.as<int32_t>()[1];
  if (e0) SAI_THROW(SAI_EINVAL, "malformed CSR input (flags 0x%x)", e0);
  h->s = s;

  h->dense_cols.alloc(&al, (size_t)s + 1);
  DBuf<int32_t> dcount(&al, (size_t)s + 1);
  hipLaunchKernelGGL(k_dense_compact, dim3(grid_for(n, NT)), dim3(NT), 0, st, n, flag.p, pos.p,
                     colcnt.p, h->dense_cols.p, dcount.p, colmap.p);
  LAUNCH_CHECK();

  DBuf<uint8_t> drop(&al, (size_t)nnz + 1);
  HIPC(hipMemsetAsync(drop.p, 0, (size_t)nnz + 1, st));
  int64_t nnz_u = 0;
  if (s > 0) {
    std::vector<int32_t> hc(s);
    HIPC(hipMemcpyAsync(hc.data(), dcount.p, sizeof(int32_t) * s, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    std::vector<int64_t> hoff(s + 1, 0);
    for (int d = 0; d < s; ++d) hoff[d + 1] = hoff[d] + hc[d];
    DBuf<int64_t> doff(&al, (size_t)s + 1);
    DBuf<int32_t> dcur(&al, (size_t)s + 1), lrow(&al, (size_t)hoff[s] + 1), lpos(&al, (size_t)hoff[s] + 1);
    HIPC(hipMemcpyAsync(doff.p, hoff.data(), sizeof(int64_t) * (s + 1), hipMemcpyHostToDevice, st));
    if (s <= GATHER_SMAX) {
      const int nbk = (int)((n + GATHER_ROWS - 1) / GATHER_ROWS);
      DBuf<int32_t> bcnt(&al, (size_t)s * nbk + 1);
      DBuf<int64_t> boff(&al, (size_t)s * nbk + 1);
      hipLaunchKernelGGL(k_dense_gather_blk, dim3(nbk), dim3(NT), 0, st, n, s, row_ptr, col_idx,
                         colmap.p, 0, bcnt.p, (const int64_t*)nullptr, lrow.p, lpos.p);
      LAUNCH_CHECK();
      exclusive_scan_i32_to_i64(bcnt.p, boff.p, (int64_t)s * nbk, al, st);
      hipLaunchKernelGGL(k_dense_gather_blk, dim3(nbk), dim3(NT), 0, st, n, s, row_ptr, col_idx,
                         colmap.p, 1, bcnt.p, (const int64_t*)boff.p, lrow.p, lpos.p);
      LAUNCH_CHECK();
    } else {
      HIPC(hipMemsetAsync(dcur.p, 0, sizeof(int32_t) * (s + 1), st));
      hipLaunchKernelGGL(k_dense_gather, dim3(grid_for(n, NT)), dim3(NT), 0, st, n, row_ptr, col_idx,
                         colmap.p, doff.p, dcur.p, lrow.p, lpos.p);
      LAUNCH_CHECK();
    }
    if (keep - 1 <= SEL_K)
      hipLaunchKernelGGL(k_dense_select_k, dim3(s), dim3(SEL_NT), 0, st, h->dense_cols.p, doff.p, dcount.p,
                         lrow.p, lpos.p, val, keep, o.rule, drop.p, err.p);
    else
      hipLaunchKernelGGL(k_dense_select, dim3(s), dim3(NT), 0, st, h->dense_cols.p, doff.p, dcount.p,
                         lrow.p, lpos.p, val, keep, o.rule, drop.p, err.p);
    LAUNCH_CHECK();
    const int e1 = read_scalar(err.p, st);
    if (e1 & ERR_ZERODIAG) SAI_THROW(SAI_EZERODIAG, "an irregular column has no diagonal entry");
    for (int d = 0; d < s; ++d) nnz_u += hc[d] - std::min<int64_t>(hc[d], keep);
  }
  const int64_t nnz_t = nnz - nnz_u;
  h->nnz_t = nnz_t;
  h->nnz_u = nnz_u;

  DBuf<int32_t> tcnt(&al, (size_t)n + 1), ucnt(&al, (size_t)n + 1);
  hipLaunchKernelGGL(k_row_counts, dim3(grid_for(n, NT)), dim3(NT), 0, st, n, row_ptr, drop.p,
                     tcnt.p, ucnt.p);
  LAUNCH_CHECK();
  h->t_row_ptr.alloc(&al, (size_t)n + 1);
  h->u_row_ptr.alloc(&al, (size_t)n + 1);
  exclusive_scan_i32(tcnt.p, h->t_row_ptr.p, n, al, st);
  exclusive_scan_i32(ucnt.p, h->u_row_ptr.p, n, al, st);
  h->t_col_idx.alloc(&al, (size_t)nnz_t + 1);
  h->t_val.alloc(&al, (size_t)nnz_t + 1);
  h->u_col.alloc(&al, (size_t)nnz_u + 1);
  h->u_val.alloc(&al, (size_t)nnz_u + 1);
  hipLaunchKernelGGL(k_row_scatter, dim3(grid_for(n, NT)), dim3(NT), 0, st, n, row_ptr, col_idx, val,
                     drop.p, colmap.p, h->t_row_ptr.p, h->t_col_idx.p, h->t_val.p, h->u_row_ptr.p,
                     h->u_col.p, h->u_val.p);
  LAUNCH_CHECK();
  {
    int32_t tot[2];
    HIPC(hipMemcpyAsync(&tot[0], h->t_row_ptr.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(&tot[1], h->u_row_ptr.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (tot[0] != nnz_t || tot[1] != nnz_u)
      SAI_THROW(SAI_EHIP, "split count mismatch (%d/%lld, %d/%lld)", tot[0], (long long)nnz_t, tot[1],
                (long long)nnz_u);
  }
  // CSC of A~
  h->t_col_ptr.alloc(&al, (size_t)n + 1);
  h->t_row_idx.alloc(&al, (size_t)nnz_t + 1);
  h->t_cval.alloc(&al, (size_t)nnz_t + 1);
  csr_transpose<double>(n, n, h->t_row_ptr.p, h->t_col_idx.p, h->t_val.p, h->t_col_ptr.p,
                        h->t_row_idx.p, h->t_cval.p, al, st);
  // structure of A (gradients are returned in A's CSR order)
  h->a_row_ptr.alloc(&al, (size_t)n + 1);
  h->a_col_idx.alloc(&al, (size_t)nnz + 1);
  HIPC(hipMemcpyAsync(h->a_row_ptr.p, row_ptr, sizeof(int32_t) * ((size_t)n + 1),
                      hipMemcpyDeviceToDevice, st));
  if (nnz > 0)
    HIPC(hipMemcpyAsync(h->a_col_idx.p, col_idx, sizeof(int32_t) * (size_t)nnz,
                        hipMemcpyDeviceToDevice, st));
  HIPC(hipStreamSynchronize(st));
}

}  // namespace sai
