// Pattern builder: J_k (pattern of column k of M) and I_k (nonzero rows of
// A~(:, J_k)) for every column, from the CSC of A~.
//
// J_k = P(A~(:,k)) or, for the static PSAI-style pattern, the structural
// P(|A~|^2 e_k) = union of P(A~(:,j)) over j in P(A~(:,k)) (Section 2.2, the
// l = 2 member of the BPSAI envelope P((I+|A|)^l)).  I_k = union of
// P(A~(:,j)) over j in J_k (Section 2, definition of L_k before (lsprob)).
//
// One wavefront (a 64-thread workgroup) per column: the candidate indices of a
// union are gathered into LDS, bitonic-sorted and de-duplicated with a ballot
// prefix (or, for small unions, an LDS hash table and a rank sort), so both
// lists come out sorted ascending.  The lists are written at offsets from cheap
// upper bounds of their lengths and then packed.
#include "sai_internal.hpp"

namespace sai {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// Gather the concatenation of P(A~(:, L[t])) for t < nL into cand[0..m); returns m
// (or -1 if it would exceed cap).  L and the scratch arrays live in LDS.
__device__ int gather_cols(const int32_t* __restrict__ cp, const int32_t* __restrict__ ri,
                           const int32_t* L, int nL, int32_t* cand, int cap, int32_t* s_start,
                           int32_t* s_off /* nL */) {
  const int l = lane_id();
  // column starts and a running prefix of the counts
  int base = 0;
  for (int t0 = 0; t0 < nL; t0 += WAVE) {
    const int t = t0 + l;
    int c = 0;
    if (t < nL) {
      const int32_t j = L[t];
      const int32_t a = cp[j];
      c = cp[j + 1] - a;
      s_start[t] = a;
    }
    // inclusive wave scan of c
    int incl = c;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      int v = __shfl_up(incl, o, WAVE);
      if (l >= o) incl += v;
    }
    if (t < nL) s_off[t] = base + incl - c;
    base += __shfl(incl, WAVE - 1, WAVE);
  }
  __syncthreads();
  if (base > cap) return -1;
  for (int f = l; f < base; f += WAVE) {
    // t = last index with s_off[t] <= f
    int lo = 0, hi = nL - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= f) lo = mid; else hi = mid - 1;
    }
    cand[f] = ri[s_start[lo] + (f - s_off[lo])];
  }
  __syncthreads();
  return base;
}

// Sort cand[0..m) ascending in place (bitonic over the next power of two) and
// remove duplicates; returns the number of unique values.
__device__ int sort_unique(int32_t* cand, int m, int cap) {
  const int l = lane_id();
  int P = 1;
  while (P < m) P <<= 1;
  if (P > cap) P = cap;  // m <= cap and cap is a power of two
  for (int i = m + l; i < P; i += WAVE) cand[i] = 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = l; t < (P >> 1); t += WAVE) {
        const int i = 2 * j * (t / j) + (t % j);
        const int q = i + j;
        const int32_t a = cand[i], b = cand[q];
        const bool up = (i & k) == 0;
        if ((a > b) == up) { cand[i] = b; cand[q] = a; }
      }
      __syncthreads();
    }
  }
  int out = 0;
  for (int c0 = 0; c0 < m; c0 += WAVE) {
    const int i = c0 + l;
    int32_t v = 0;
    bool keep = false;
    if (i < m) {
      v = cand[i];
      keep = (i == 0) || (cand[i - 1] != v);
    }
    const unsigned long long bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << l) - 1ull));
    __syncthreads();
    if (keep) cand[out + before] = v;
    out += __popcll(bal);
    __syncthreads();
  }
  return out;
}

// Fast path of sort_unique for small unions (the common case for regular sparse
// A~): de-duplicate through an LDS hash table (linear probing, atomicCAS), then
// sort the <= 64 distinct values by rank (one value per lane, ranks from a
// 64-step broadcast loop) and write them in order.  Falls back to the bitonic
// sort when there are more than 64 distinct values or more than 512 candidates.
constexpr int HT = 256;
constexpr int32_t HT_EMPTY = 0x7fffffff;
// |J_k| held by the large variants of the pattern and row-set kernels (the
// large column-solver limits)
constexpr int CAPJ_L = 512;

__device__ int sort_unique_fast(int32_t* cand, int m, int cap, int32_t* ht) {
  const int l = lane_id();
  if (m == 0) return 0;
  if (m > 512) return sort_unique(cand, m, cap);
  for (int i = l; i < HT; i += WAVE) ht[i] = HT_EMPTY;
  __syncthreads();
  int fresh = 0;
  for (int i = l; i < m; i += WAVE) {
    const int32_t v = cand[i];
    unsigned h = ((unsigned)v * 2654435761u) >> 24;
    bool placed = false;
    for (int probe = 0; probe < HT; ++probe) {  // a full table ends the probing
      const int32_t old = atomicCAS(&ht[h], HT_EMPTY, v);
      if (old == HT_EMPTY) { ++fresh; placed = true; break; }
      if (old == v) { placed = true; break; }
      h = (h + 1) & (HT - 1);
    }
    if (!placed) fresh += HT;  // forces the fallback below
  }
  const int nu = wave_sum(fresh);
  __syncthreads();
  if (nu > WAVE) return sort_unique(cand, m, cap);
  // compact the occupied slots into cand[0..nu) (the candidates are no longer
  // needed), one value per lane
  int base = 0;
  for (int s0 = 0; s0 < HT; s0 += WAVE) {
    const int32_t hv = ht[s0 + l];
    const bool occ = hv != HT_EMPTY;
    const unsigned long long bal = __ballot(occ);
    if (occ) cand[base + __popcll(bal & ((l == 0) ? 0ull : (~0ull >> (64 - l))))] = hv;
    base += __popcll(bal);
  }
  __syncthreads();
  const int32_t u = l < nu ? cand[l] : HT_EMPTY;
  // rank of u among the nu values (distinct), then ordered write
  int rank = 0;
  for (int t = 0; t < nu; ++t) {
    const int32_t o = __shfl(u, t, WAVE);
    rank += (o < u) ? 1 : 0;
  }
  __syncthreads();
  if (l < nu) cand[rank] = u;
  __syncthreads();
  return nu;
}

// mode 0: counts only; 1: lists at jptr/iptr; 2: lists at jptr/iptr and counts.
// A column whose unions overflow the capacities gets cntJ = -1 (modes 0, 2).
// Work item b < nwork is column list[b] (or column b when list is NULL).
template <int CAP, int CAPJ = 256>
__global__ void __launch_bounds__(64) k_pattern(int32_t nwork, int kind, const int32_t* __restrict__ cp,
                                                const int32_t* __restrict__ ri, int mode,
                                                const int32_t* __restrict__ list,
                                                int32_t* __restrict__ cntJ, int32_t* __restrict__ cntI,
                                                const int64_t* __restrict__ jptr,
                                                int32_t* __restrict__ jout,
                                                const int64_t* __restrict__ iptr,
                                                int32_t* __restrict__ iout, int* __restrict__ nover) {
  static_assert(CAPJ >= HT, "the hash table reuses the gather scratch");
  __shared__ int32_t cand[CAP];
  __shared__ int32_t sJ[CAPJ];
  // gather scratch; the hash table of a union reuses s_start once the
  // candidates are gathered
  __shared__ int32_t s_start[CAPJ];
  __shared__ int32_t s_off[CAPJ];
  int32_t* const ht = s_start;
  const int l = lane_id();
  for (int64_t b = blockIdx.x; b < nwork; b += gridDim.x) {
    const int64_t k = list ? (int64_t)list[b] : b;
    int nJ;
    // ---- J_k
    const int32_t a0 = cp[k], c0 = cp[k + 1] - cp[k];
    if (kind == SAI_PAT_A2) {
      // L = P(A~(:,k)), kept in sJ temporarily
      if (c0 > CAPJ) { if (l == 0 && mode != 1) { cntJ[k] = -1; atomicAdd(nover, 1); } continue; }
      for (int t = l; t < c0; t += WAVE) sJ[t] = ri[a0 + t];
      __syncthreads();
      int m = gather_cols(cp, ri, sJ, c0, cand, CAP, s_start, s_off);
      if (m < 0) { if (l == 0 && mode != 1) { cntJ[k] = -1; atomicAdd(nover, 1); } __syncthreads(); continue; }
      nJ = sort_unique_fast(cand, m, CAP, ht);
      if (nJ > CAPJ) { if (l == 0 && mode != 1) { cntJ[k] = -1; atomicAdd(nover, 1); } __syncthreads(); continue; }
      for (int t = l; t < nJ; t += WAVE) sJ[t] = cand[t];
      __syncthreads();
    } else {
      if (c0 > CAPJ) { if (l == 0 && mode != 1) { cntJ[k] = -1; atomicAdd(nover, 1); } continue; }
      nJ = c0;
      for (int t = l; t < nJ; t += WAVE) sJ[t] = ri[a0 + t];
      __syncthreads();
    }
    // ---- I_k
    int m = gather_cols(cp, ri, sJ, nJ, cand, CAP, s_start, s_off);
    if (m < 0) { if (l == 0 && mode != 1) { cntJ[k] = -1; atomicAdd(nover, 1); } __syncthreads(); continue; }
    const int nI = sort_unique_fast(cand, m, CAP, ht);
    if (mode != 1) {
      if (l == 0) { cntJ[k] = nJ; cntI[k] = nI; }
    }
    if (mode != 0) {
      const int64_t jo = jptr[k], io = iptr[k];
      for (int t = l; t < nJ; t += WAVE) jout[jo + t] = sJ[t];
      for (int t = l; t < nI; t += WAVE) iout[io + t] = cand[t];
    }
    __syncthreads();
  }
}

// Upper bounds of |J_k| and |I_k| from column lengths only (no de-duplication):
// w[j] = sum of |P(A~(:,i))| over i in P(A~(:,j)); for the static pattern
// P(|A~|^2 e_k), |J_k| <= sum_{j in P(A~(:,k))} |P(A~(:,j))| and
// |I_k| <= sum_{j in P(A~(:,k))} w[j]; for J_k = P(A~(:,k)), |I_k| <= w[k].
__global__ void k_pat_w(int32_t n, const int32_t* __restrict__ cp, const int32_t* __restrict__ ri,
                        int64_t* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  int64_t s = 0;
  for (int32_t e = cp[j]; e < cp[j + 1]; ++e) {
    const int32_t i = ri[e];
    s += cp[i + 1] - cp[i];
  }
  w[j] = s;
}

__global__ void k_pat_ub(int32_t n, int kind, const int32_t* __restrict__ cp,
                         const int32_t* __restrict__ ri, const int64_t* __restrict__ w,
                         int64_t* __restrict__ ubJ, int64_t* __restrict__ ubI) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  if (kind == SAI_PAT_A2) {
    int64_t sj = 0, si = 0;
    for (int32_t e = cp[k]; e < cp[k + 1]; ++e) {
      const int32_t j = ri[e];
      sj += cp[j + 1] - cp[j];
      si += w[j];
    }
    ubJ[k] = sj;
    ubI[k] = si;
  } else {
    ubJ[k] = cp[k + 1] - cp[k];
    ubI[k] = w[k];
  }
}

// Copy the lists written at upper-bound offsets (src_ptr[k], length cnt[k]) to
// their packed places dst_ptr[k], coalesced, 16 lanes per list (four lists per
// wavefront): the lists here hold tens of entries (100^3 matrix: 0.52 ms with
// 64 lanes per list, 0.39 with 32, 0.34 with 16).
__global__ void __launch_bounds__(256) k_pack_lists(int32_t n, const int64_t* __restrict__ src_ptr,
                                                    const int32_t* __restrict__ src,
                                                    const int64_t* __restrict__ dst_ptr,
                                                    int32_t* __restrict__ dst) {
  constexpr int LPC = 16;
  const int l = threadIdx.x % LPC;
  for (int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPC; k < n;
       k += (int64_t)gridDim.x * (256 / LPC)) {
    const int64_t a = src_ptr[k], b = dst_ptr[k];
    const int c = (int)(dst_ptr[k + 1] - b);
    for (int t = l; t < c; t += LPC) dst[b + t] = src[a + t];
  }
}

// I_k = union of P(A~(:, j)) over the given J_k (count pass: mode 0, fill: mode 1).
template <int CAP, int CAPJ = 256>
__global__ void __launch_bounds__(64) k_rows_of(int32_t nwork, const int32_t* __restrict__ list,
                                                const int32_t* __restrict__ cp,
                                                const int32_t* __restrict__ ri,
                                                const int64_t* __restrict__ jptr,
                                                const int32_t* __restrict__ jidx, int mode,
                                                int32_t* __restrict__ cntI,
                                                const int64_t* __restrict__ iptr,
                                                int32_t* __restrict__ iout, int* __restrict__ nover) {
  static_assert(CAPJ >= HT, "the hash table reuses the gather scratch");
  __shared__ int32_t cand[CAP];
  __shared__ int32_t sJ[CAPJ];
  // gather scratch; the hash table of a union reuses s_start once the
  // candidates are gathered
  __shared__ int32_t s_start[CAPJ];
  __shared__ int32_t s_off[CAPJ];
  int32_t* const ht = s_start;
  const int l = lane_id();
  // a column that overflows CAP gets cntI = -1 in the counting pass (mode 0)
  // and is skipped in the writing pass (the larger variant redoes it)
  for (int64_t b = blockIdx.x; b < nwork; b += gridDim.x) {
    const int64_t k = list ? (int64_t)list[b] : b;
    const int64_t j0 = jptr[k];
    const int nJ = (int)(jptr[k + 1] - j0);
    if (nJ > CAPJ) { if (l == 0 && mode == 0) { cntI[k] = -1; atomicAdd(nover, 1); } continue; }
    for (int t = l; t < nJ; t += WAVE) sJ[t] = jidx[j0 + t];
    __syncthreads();
    const int m = gather_cols(cp, ri, sJ, nJ, cand, CAP, s_start, s_off);
    if (m < 0) { if (l == 0 && mode == 0) { cntI[k] = -1; atomicAdd(nover, 1); } __syncthreads(); continue; }
    const int nI = sort_unique_fast(cand, m, CAP, ht);
    if (mode == 0) {
      if (l == 0) cntI[k] = nI;
    } else {
      const int64_t io = iptr[k];
      for (int t = l; t < nI; t += WAVE) iout[io + t] = cand[t];
    }
    __syncthreads();
  }
}

// The columns with cnt < 0, in unspecified order (at most cap of them kept),
// and their number.
__global__ void __launch_bounds__(256) k_list_neg(int32_t n, const int32_t* __restrict__ cnt,
                                                  int32_t* __restrict__ list, int cap,
                                                  int* __restrict__ count) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool neg = k < n && cnt[k] < 0;
  const int slot = block_slot<1>(count, neg ? 0 : -1);
  if (neg && slot < cap) list[slot] = (int32_t)k;
}

void rows_of_patterns(const sai_split_s* sp, hipStream_t st, const Allocator& al,
                      const DBuf<int64_t>& jptr, const DBuf<int32_t>& jidx, DBuf<int64_t>& iptr,
                      DBuf<int32_t>& iidx, DBuf<int32_t>& cntI) {
  const int32_t n = sp->n;
  // every column through the 5 KB kernel (eight waves per SIMD); the few whose
  // candidate lists overflow it are redone by the 32 KB one over a list
  constexpr int CAP_S = 512, CAP_L = 8192;
  cntI.alloc(&al, (size_t)n + 1);
  DBuf<int> nover(&al, 2);
  HIPC(hipMemsetAsync(nover.p, 0, 2 * sizeof(int), st));
  const unsigned grid = (unsigned)std::min<int64_t>(n, 1 << 20);
  const int32_t* cp = sp->t_col_ptr.p;
  const int32_t* ri = sp->t_row_idx.p;
  hipLaunchKernelGGL((k_rows_of<CAP_S>), dim3(grid), dim3(64), 0, st, n, (const int32_t*)nullptr, cp, ri,
                     jptr.p, jidx.p, 0, cntI.p, (const int64_t*)nullptr, (int32_t*)nullptr, nover.p);
  LAUNCH_CHECK();
  const int nbig = read_scalar(nover.p, st);
  DBuf<int32_t> list;
  if (nbig > 0) {
    list.alloc(&al, (size_t)nbig);
    HIPC(hipMemsetAsync(nover.p, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_list_neg, dim3(grid_for(n, 256)), dim3(256), 0, st, n, cntI.p, list.p, nbig,
                       nover.p + 1);
    LAUNCH_CHECK();
    if (read_scalar(nover.p + 1, st) != nbig)
      SAI_THROW(SAI_EHIP, "row-set overflow list: %d columns listed, %d counted",
                read_scalar(nover.p + 1, st), nbig);
    hipLaunchKernelGGL((k_rows_of<CAP_L, CAPJ_L>), dim3(std::min(nbig, 1 << 20)), dim3(64), 0, st, nbig,
                       (const int32_t*)list.p, cp, ri, jptr.p, jidx.p, 0, cntI.p, (const int64_t*)nullptr,
                       (int32_t*)nullptr, nover.p);
    LAUNCH_CHECK();
    if (read_scalar(nover.p, st) > 0)
      SAI_THROW(SAI_ETOOBIG, "a pattern exceeds %d indices or a row set I_k %d candidate indices", CAPJ_L,
                CAP_L);
  }
  iptr.alloc(&al, (size_t)n + 1);
  exclusive_scan_i32_to_i64(cntI.p, iptr.p, n, al, st);
  const int64_t tot = read_scalar(iptr.p + n, st);
  iidx.alloc(&al, (size_t)tot + 1);
  hipLaunchKernelGGL((k_rows_of<CAP_S>), dim3(grid), dim3(64), 0, st, n, (const int32_t*)nullptr, cp, ri,
                     jptr.p, jidx.p, 1, cntI.p, (const int64_t*)iptr.p, iidx.p, nover.p);
  LAUNCH_CHECK();
  if (nbig > 0) {
    hipLaunchKernelGGL((k_rows_of<CAP_L, CAPJ_L>), dim3(std::min(nbig, 1 << 20)), dim3(64), 0, st, nbig,
                       (const int32_t*)list.p, cp, ri, jptr.p, jidx.p, 1, cntI.p, (const int64_t*)iptr.p,
                       iidx.p, nover.p);
    LAUNCH_CHECK();
  }
}


// Sizes, offsets and lists of J_k and I_k.  jptr/iptr get n+1 entries.
// One union pass: the lists are written at offsets from upper bounds of their
// lengths (no de-duplication needed for the bounds), with their exact lengths,
// then packed to the offsets of the exact lengths.
void build_patterns(const sai_split_s* sp, int kind, hipStream_t st, const Allocator& al,
                    DBuf<int64_t>& jptr, DBuf<int32_t>& jidx, DBuf<int64_t>& iptr,
                    DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ, DBuf<int32_t>& cntI) {
  const int32_t n = sp->n;
  const int32_t* cp = sp->t_col_ptr.p;
  const int32_t* ri = sp->t_row_idx.p;
  cntJ.alloc(&al, (size_t)n + 1);
  cntI.alloc(&al, (size_t)n + 1);
  DBuf<int> nover(&al, 2);
  HIPC(hipMemsetAsync(nover.p, 0, 2 * sizeof(int), st));
  const unsigned grid = (unsigned)std::min<int64_t>(n, 1 << 20);
  // CAP_S = 512 keeps the small kernel within 5 KB of LDS (32 workgroups per CU)
  constexpr int CAP_S = 512, CAP_L = 8192;
  DBuf<int64_t> ujo(&al, (size_t)n + 1), uio(&al, (size_t)n + 1);
  DBuf<int32_t> tJ, tI;
  {
    SAI_PROF("pattern_bounds", st);
    DBuf<int64_t> w(&al, (size_t)n + 1), ubJ(&al, (size_t)n + 1), ubI(&al, (size_t)n + 1);
    hipLaunchKernelGGL(k_pat_w, dim3(grid_for(n, 256)), dim3(256), 0, st, n, cp, ri, w.p);
    hipLaunchKernelGGL(k_pat_ub, dim3(grid_for(n, 256)), dim3(256), 0, st, n, kind, cp, ri, w.p, ubJ.p,
                       ubI.p);
    LAUNCH_CHECK();
    exclusive_scan_i64(ubJ.p, ujo.p, n, al, st);
    exclusive_scan_i64(ubI.p, uio.p, n, al, st);
    int64_t ub[2];
    HIPC(hipMemcpyAsync(&ub[0], ujo.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(&ub[1], uio.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    tJ.alloc(&al, (size_t)ub[0] + 1);
    tI.alloc(&al, (size_t)ub[1] + 1);
  }
  {
    SAI_PROF("pattern_fill", st);
    hipLaunchKernelGGL((k_pattern<CAP_S>), dim3(grid), dim3(64), 0, st, n, kind, cp, ri, 2,
                       (const int32_t*)nullptr, cntJ.p, cntI.p, (const int64_t*)ujo.p, tJ.p,
                       (const int64_t*)uio.p, tI.p, nover.p);
    LAUNCH_CHECK();
    const int nbig = read_scalar(nover.p, st);
    if (nbig > 0) {
      // columns whose unions overflow the small kernel are redone by the large
      // one, over a list of just those columns
      DBuf<int32_t> list(&al, (size_t)nbig);
      HIPC(hipMemsetAsync(nover.p, 0, 2 * sizeof(int), st));
      hipLaunchKernelGGL(k_list_neg, dim3(grid_for(n, 256)), dim3(256), 0, st, n, cntJ.p, list.p, nbig,
                         nover.p + 1);
      LAUNCH_CHECK();
      // every column of the first pass got its count or -1, one -1 per overflow
      if (read_scalar(nover.p + 1, st) != nbig)
        SAI_THROW(SAI_EHIP, "pattern overflow list: %d columns listed, %d counted",
                  read_scalar(nover.p + 1, st), nbig);
      hipLaunchKernelGGL((k_pattern<CAP_L, CAPJ_L>), dim3(std::min(nbig, 1 << 20)), dim3(64), 0, st, nbig, kind,
                         cp, ri, 2, (const int32_t*)list.p, cntJ.p, cntI.p, (const int64_t*)ujo.p, tJ.p,
                         (const int64_t*)uio.p, tI.p, nover.p);
      LAUNCH_CHECK();
      if (read_scalar(nover.p, st) > 0)
        SAI_THROW(SAI_ETOOBIG, "a pattern exceeds %d indices or its unions %d candidate indices", CAPJ_L,
                  CAP_L);
    }
  }
  SAI_PROF("pattern_pack", st);
  jptr.alloc(&al, (size_t)n + 1);
  iptr.alloc(&al, (size_t)n + 1);
  exclusive_scan_i32_to_i64(cntJ.p, jptr.p, n, al, st);
  exclusive_scan_i32_to_i64(cntI.p, iptr.p, n, al, st);
  int64_t tot[2];
  HIPC(hipMemcpyAsync(&tot[0], jptr.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(&tot[1], iptr.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  jidx.alloc(&al, (size_t)tot[0] + 1);
  iidx.alloc(&al, (size_t)tot[1] + 1);
  const unsigned pgrid = grid_for((int64_t)n * 16, 256, 8192);
  hipLaunchKernelGGL(k_pack_lists, dim3(pgrid), dim3(256), 0, st, n, ujo.p, tJ.p, jptr.p, jidx.p);
  hipLaunchKernelGGL(k_pack_lists, dim3(pgrid), dim3(256), 0, st, n, uio.p, tI.p, iptr.p, iidx.p);
  LAUNCH_CHECK();
}

}  // namespace sai
