// Standalone gather of the column least-squares blocks (Section 2, (lsprob)):
// for every column k with pattern J_k and row set I_k (the nonzero rows of
// A~(:, J_k)), the dense block A~(I_k, J_k) is written column-major at element
// offset blk_off[k] of the output (|I_k| rows, leading dimension |I_k|).  The
// column solvers gather the same blocks into registers or LDS and factor them
// at once; this kernel performs only that gather, so that its memory traffic
// can be measured and so that the blocks can be handed to other solvers.
//
// One wavefront per column.  When |J_k| <= 64, |I_k| <= CAPI and the gathered
// entries fit CAPE, the wavefront stages the rows of I_k and the entries (row,
// value) of the columns A~(:, J_k) in LDS (lane c reads the CSC range of
// column J_k[c]; a wavefront scan turns the column lengths into offsets, and
// the entries are then copied 64 at a time), and every output element (r, c)
// is found by a binary search of I_k[r] among column c's staged rows (0 if
// absent).  Each lane produces four consecutive elements of the column-major
// block and writes them with one 16-byte store (the first and last partial
// groups element by element), so a column costs a few dependent loads and
// about |I_k| |J_k| / 256 stores.  Other blocks are filled element by element
// from the CSC arrays in global memory.
#include "sai_internal.hpp"

namespace sai {
namespace {

constexpr int GNT = 256;              // 4 wavefronts per workgroup, one column each
constexpr int GW = GNT / WAVE;
constexpr int CAPI = 256;             // rows of I_k staged in LDS
constexpr int CAPE = 256;             // gathered entries staged in LDS (4.6 KB per wavefront)

__global__ void k_gather_sizes(int32_t n, const int64_t* __restrict__ jptr, const int64_t* __restrict__ iptr,
                               int64_t* __restrict__ sz) {
  const int64_t k = (int64_t)blockIdx.x * GNT + threadIdx.x;
  if (k < n) sz[k] = (jptr[k + 1] - jptr[k]) * (iptr[k + 1] - iptr[k]);
}

__device__ __forceinline__ int find_row(const int32_t* a, int m, int32_t x) {
  int lo = 0, hi = m;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;  // a[lo] == x: x is a row of A~(:, J_k), hence in I_k
}

// A~(I_k[r], J_k[c]) from the staged entries: row I_k[r] among column c's rows
template <class T>
__device__ __forceinline__ T elem_rc(int r, int c, const int32_t* sr, const int32_t* so, const int32_t* er,
                                     const double* ev) {
  const int32_t row = sr[r];
  int lo = so[c], hi = so[c + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (er[mid] < row) lo = mid + 1; else hi = mid;
  }
  return (lo < so[c + 1] && er[lo] == row) ? (T)ev[lo] : (T)0;
}

template <class T>
__device__ __forceinline__ T elem(int t, int nI, const int32_t* sr, const int32_t* so, const int32_t* er,
                                  const double* ev) {
  const int c = t / nI;
  return elem_rc<T>(t - c * nI, c, sr, so, er, ev);
}

// V consecutive elements t0 .. t0 + V - 1 of the column-major block
template <class T, int V>
__device__ __forceinline__ void elems(int t0, int nI, const int32_t* sr, const int32_t* so, const int32_t* er,
                                      const double* ev, T* v) {
  int c = t0 / nI, r = t0 - c * nI;
#pragma unroll
  for (int u = 0; u < V; ++u) {
    v[u] = elem_rc<T>(r, c, sr, so, er, ev);
    if (++r == nI) { r = 0; ++c; }
  }
}

template <class T>
__global__ void __launch_bounds__(GNT) k_gather(int32_t n, const int32_t* __restrict__ cp,
                                                const int32_t* __restrict__ ri, const double* __restrict__ cv,
                                                const int64_t* __restrict__ jptr, const int32_t* __restrict__ jidx,
                                                const int64_t* __restrict__ iptr, const int32_t* __restrict__ iidx,
                                                const int64_t* __restrict__ boff, T* __restrict__ out) {
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte store
  __shared__ int32_t srow[GW][CAPI];
  __shared__ int32_t soff[GW][WAVE + 1];
  __shared__ int32_t sbeg[GW][WAVE];
  __shared__ int32_t erow[GW][CAPE];
  __shared__ double eval[GW][CAPE];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  int32_t* sr = srow[w];
  int32_t* so = soff[w];
  int32_t* sb = sbeg[w];
  int32_t* er = erow[w];
  double* ev = eval[w];
  for (int64_t k = (int64_t)blockIdx.x * GW + w; k < n; k += (int64_t)gridDim.x * GW) {
    const int64_t ja = jptr[k], ia = iptr[k];
    const int nJ = (int)(jptr[k + 1] - ja), nI = (int)(iptr[k + 1] - ia);
    const int64_t o = boff[k];
    const int64_t ne = (int64_t)nJ * nI;
    // the rows of I_k are loaded first, so that their latency overlaps the
    // column-pointer loads below (kept in registers until the path is known)
    constexpr int RI = CAPI / WAVE;
    int32_t irow[RI];
#pragma unroll
    for (int u = 0; u < RI; ++u) {
      const int t = lane + u * WAVE;
      irow[u] = (nI <= CAPI && t < nI) ? iidx[ia + t] : 0;
    }
    int32_t beg = 0, len = 0;
    if (lane < nJ && nJ <= WAVE) {
      const int32_t j = jidx[ja + lane];
      beg = cp[j];
      len = cp[j + 1] - beg;
    }
    int32_t incl = len;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      const int32_t t = __shfl_up(incl, d, WAVE);
      if (lane >= d) incl += t;
    }
    const int32_t tot = __shfl(incl, WAVE - 1, WAVE);
    if (nJ <= WAVE && nI <= CAPI && tot <= CAPE) {
      so[lane + 1] = incl;
      if (lane == 0) so[0] = 0;
      sb[lane] = beg;
#pragma unroll
      for (int u = 0; u < RI; ++u) {
        const int t = lane + u * WAVE;
        if (t < nI) sr[t] = irow[u];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // entry f of column c (so[c] <= f < so[c + 1]) is CSC entry beg_c + f - so[c];
      // a lane's (up to CAPE / WAVE) entries are located first, then all their
      // loads issued together
      constexpr int RE = CAPE / WAVE;
      int32_t ee[RE];
#pragma unroll
      for (int u = 0; u < RE; ++u) {
        const int32_t f = lane + u * WAVE;
        ee[u] = -1;
        if (f < tot) {
          int lo = 0, hi = nJ - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (so[mid] <= f) lo = mid; else hi = mid - 1;
          }
          ee[u] = sb[lo] + (f - so[lo]);
        }
      }
      int32_t rr[RE];
      double vv[RE];
#pragma unroll
      for (int u = 0; u < RE; ++u) {
        rr[u] = ee[u] >= 0 ? ri[ee[u]] : 0;
        vv[u] = ee[u] >= 0 ? cv[ee[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RE; ++u) {
        const int32_t f = lane + u * WAVE;
        if (f < tot) {
          er[f] = rr[u];
          ev[f] = vv[u];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // head (until out + o + t is 16-byte aligned), 16-byte groups, tail
      const int head = (int)((V - (int)(o % V)) % V);
      const int h = (int)(head < ne ? head : ne);
      if (lane < h) out[o + lane] = elem<T>(lane, nI, sr, so, er, ev);
      const int nv = (int)((ne - h) / V);
      for (int g = lane; g < nv; g += WAVE) {
        const int t0 = h + g * V;
        T v[V];
        elems<T, V>(t0, nI, sr, so, er, ev, v);
        // the blocks are written once and not read back here: non-temporal
        // stores keep them from displacing the CSC entries that neighbouring
        // columns gather again
        if constexpr (V == 4) {
          typedef float f4v __attribute__((ext_vector_type(4)));
          const f4v q = {v[0], v[1], v[2], v[3]};
          __builtin_nontemporal_store(q, reinterpret_cast<f4v*>(out + o + t0));
        } else {
          typedef double d2v __attribute__((ext_vector_type(2)));
          const d2v q = {v[0], v[1]};
          __builtin_nontemporal_store(q, reinterpret_cast<d2v*>(out + o + t0));
        }
      }
      for (int t = h + nv * V + lane; t < (int)ne; t += WAVE) out[o + t] = elem<T>(t, nI, sr, so, er, ev);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      // element (r, c) = A~(I[r], J[c]): search row I[r] among column J[c]'s rows
      for (int64_t t = lane; t < ne; t += WAVE) {
        const int c = (int)(t / nI), r = (int)(t % nI);
        const int32_t j = jidx[ja + c], row = iidx[ia + r];
        const int32_t e0 = cp[j], e1 = cp[j + 1];
        int lo = e0, hi = e1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (ri[mid] < row) lo = mid + 1; else hi = mid;
        }
        out[o + t] = (lo < e1 && ri[lo] == row) ? (T)cv[lo] : (T)0;
      }
    }
  }
}

}  // namespace

void gather_offsets(const sai_precond_s* pc, int64_t* blk_off, int64_t* total, hipStream_t st) {
  if (!pc->j_ptr.p || !pc->i_ptr.p)
    SAI_THROW(SAI_EINVAL, "the preconditioner was built without keep_lists: no J_k, I_k to gather");
  const Allocator al{pc->al.a, st};
  const int32_t n = pc->n;
  DBuf<int64_t> sz(&al, (size_t)n + 1);
  hipLaunchKernelGGL(k_gather_sizes, dim3(grid_for(n, GNT)), dim3(GNT), 0, st, n, pc->j_ptr.p, pc->i_ptr.p,
                     sz.p);
  LAUNCH_CHECK();
  exclusive_scan_i64(sz.p, blk_off, n, al, st);
  if (total) *total = read_scalar(blk_off + n, st);
  HIPC(hipStreamSynchronize(st));
}

void gather_blocks(const sai_split_s* sp, const sai_precond_s* pc, int precision, const int64_t* blk_off,
                   void* blocks, hipStream_t st) {
  if (!pc->j_ptr.p || !pc->i_ptr.p)
    SAI_THROW(SAI_EINVAL, "the preconditioner was built without keep_lists: no J_k, I_k to gather");
  if (precision != SAI_FP32 && precision != SAI_FP64) SAI_THROW(SAI_EINVAL, "bad precision");
  if (pc->n != sp->n) SAI_THROW(SAI_EINVAL, "split and preconditioner sizes differ");
  const int32_t n = sp->n;
  SAI_PROF(precision == SAI_FP32 ? "gather_f32" : "gather_f64", st);
  // one workgroup per four columns (a persistent grid that walks the columns
  // was slower: 13.0 against 10.1 ms on the 160^3 workload)
  const unsigned grid = grid_for(((int64_t)n + GW - 1) / GW, 1, 1u << 20);
  if (precision == SAI_FP32)
    hipLaunchKernelGGL((k_gather<float>), dim3(grid), dim3(GNT), 0, st, n, sp->t_col_ptr.p, sp->t_row_idx.p,
                       sp->t_cval.p, pc->j_ptr.p, pc->j_idx.p, pc->i_ptr.p, pc->i_idx.p, blk_off,
                       (float*)blocks);
  else
    hipLaunchKernelGGL((k_gather<double>), dim3(grid), dim3(GNT), 0, st, n, sp->t_col_ptr.p, sp->t_row_idx.p,
                       sp->t_cval.p, pc->j_ptr.p, pc->j_idx.p, pc->i_ptr.p, pc->i_idx.p, blk_off,
                       (double*)blocks);
  LAUNCH_CHECK();
  HIPC(hipStreamSynchronize(st));
}

}  // namespace sai
