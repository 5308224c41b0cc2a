// Build of M: patterns, column least squares, dropping and assembly.
//
// After every m_k is computed on its pattern J_k, entries with |m_jk| <= tol_k
// are dropped (Section 2.2, PSAI(tol), (tolk)): tol_k = tau (absolute) or
// delta / (|J_k| * ||A~||_1); the entry of largest magnitude of each column is
// always kept.  M is assembled in CSC (column k = m_k; this is the CSR of M^T
// used by the adjoint) and transposed once to CSR for the forward products.
#include "sai_internal.hpp"

namespace sai {

// defined in other translation units
void build_patterns(const sai_split_s* sp, int kind, hipStream_t st, const Allocator& al,
                    DBuf<int64_t>& jptr, DBuf<int32_t>& jidx, DBuf<int64_t>& iptr,
                    DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ, DBuf<int32_t>& cntI);
template <class T>
int solve_columns(const sai_split_s* sp, const int64_t* jptr, const int32_t* jidx,
                  const int64_t* iptr, const int32_t* iidx, const int32_t* cntJ,
                  const int32_t* cntI, int maxI, int maxJ, T* mout, double* res,
                  int64_t* bucket_cols, const Allocator& al, hipStream_t st);
template <class V>
void csr_transpose(int32_t nrows, int32_t ncols, const int32_t* rp, const int32_t* ci, const V* v,
                   int32_t* cp, int32_t* ri, V* cv, const Allocator& al, hipStream_t st);
void psai_patterns(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st,
                   const Allocator& al, DBuf<int64_t>& jptr, DBuf<int32_t>& jidx,
                   DBuf<int64_t>& iptr, DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ,
                   DBuf<int32_t>& cntI, DBuf<double>& mval, DBuf<double>& res, int* l_m);
void spai_patterns(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st,
                   const Allocator& al, DBuf<int64_t>& jptr, DBuf<int32_t>& jidx,
                   DBuf<int64_t>& iptr, DBuf<int32_t>& iidx, DBuf<int32_t>& cntJ,
                   DBuf<int32_t>& cntI, int* l_m);

namespace {

constexpr int NT = 256;

// max |I_k|, max |J_k| and (stats) the number of columns with residual > delta;
// reduced per wavefront first, then one atomic per wavefront
__device__ __forceinline__ int wmax_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wsum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(NT) k_stats(int32_t n, const int32_t* cntJ, const int32_t* cntI,
                                              const double* res, double delta,
                                              int* out /* maxI, maxJ, n_c */) {
  int mi = 0, mj = 0, nc = 0;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT) {
    mi = max(mi, cntI[k]);
    mj = max(mj, cntJ[k]);
    if (res && res[k] > delta) ++nc;
  }
  __shared__ int red[3][NT / 64];
  mi = wmax_i(mi);
  mj = wmax_i(mj);
  nc = wsum_i(nc);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = mi;
    red[1][w] = mj;
    red[2][w] = nc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NT / 64; ++q) {
      mi = max(mi, red[0][q]);
      mj = max(mj, red[1][q]);
      nc += red[2][q];
    }
    atomicMax(&out[0], mi);
    atomicMax(&out[1], mj);
    if (nc) atomicAdd(&out[2], nc);
  }
}

// ||A~||_1 = max_j sum_i |a_ij|; stored as the bit pattern of a non-negative double,
// whose integer order equals its numeric order, so atomicMax is exact.
__global__ void k_norm1(int32_t n, const int32_t* cp, const double* cv, unsigned long long* out) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int32_t e = cp[j]; e < cp[j + 1]; ++e) s += fabs(cv[e]);
  atomicMax(out, (unsigned long long)__double_as_longlong(s));
}

template <class T>
__global__ void k_to_type(int64_t m, const double* __restrict__ in, T* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (int64_t)gridDim.x * NT)
    out[i] = (T)in[i];
}

// Dropping (Section 2.2): entries of the computed column m_k with |m_jk| <= thr
// are removed (thr = tau, or (tolk) delta / (|J_k| ||A~||_1)); the entry of
// largest magnitude (the first of equals) is always kept.  16 lanes per column
// (four columns per wavefront) read the column coalesced; the kept entries keep
// their order (ballot prefix counts).  COUNT: number kept per column; else the
// kept (row, value) pairs are written from colp[k] on.  The COUNT pass also
// counts, into *nearc, the entries other than the always-kept one with
// | |m_jk| - thr | <= eta ||m_k|| / (1 - eta): an entry whose decision differs
// from that on a reference column m' with ||m_k - m'|| <= eta ||m'|| lies
// within |m_jk - m'_j| <= eta ||m'|| of thr, so these are the only decisions
// that a column accurate to eta can settle differently.
template <class T, bool COUNT>
__global__ void __launch_bounds__(NT) k_drop(int32_t n, const int64_t* __restrict__ jptr,
                                             const int32_t* __restrict__ jidx, const T* __restrict__ m,
                                             int mode, double tau, double delta, double norm1,
                                             int32_t* __restrict__ cnt, const int32_t* __restrict__ colp,
                                             int32_t* __restrict__ rowi, T* __restrict__ cval,
                                             double eta, unsigned long long* __restrict__ nearc) {
  constexpr int G = 16;  // lanes per column (four columns per wavefront)
  const int lane = threadIdx.x & 63, gi = lane & (G - 1), gbase = lane & (64 - G);
  const int64_t k = ((int64_t)blockIdx.x * NT + threadIdx.x) / G;
  const bool valid = k < n;
  const int64_t a = valid ? jptr[k] : 0, b = valid ? jptr[k + 1] : 0;
  const int nj = (int)(b - a);
  double thr = -1.0;
  if (mode == SAI_DROP_ABS) thr = tau;
  else if (mode == SAI_DROP_TOLK) thr = delta / ((double)nj * norm1);
  // largest magnitude, first index among equals; the column's squared norm
  double vmax = -1.0, ss = 0.0;
  int64_t amax = INT64_MAX;
  for (int64_t e = a + gi; e < b; e += G) {
    const double v = fabs((double)m[e]);
    if (COUNT) ss += v * v;
    if (v > vmax) { vmax = v; amax = e; }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const double ov = __shfl_xor(vmax, o, 64);
    const int64_t oa = __shfl_xor(amax, o, 64);
    if (COUNT) ss += __shfl_xor(ss, o, 64);
    if (ov > vmax || (ov == vmax && oa < amax)) { vmax = ov; amax = oa; }
  }
  const double band = eta * sqrt(ss) / (1.0 - eta);
  int32_t o = COUNT ? 0 : (valid ? colp[k] : 0);
  int nnear = 0;
  for (int64_t off = 0; __any(off < nj); off += G) {
    const int64_t e = a + off + gi;
    const double av = e < b ? fabs((double)m[e]) : 0.0;
    const bool kf = e < b && (av > thr || e == amax);
    if (COUNT && e < b && e != amax && thr > 0.0 && fabs(av - thr) <= band) ++nnear;
    const uint32_t gm = (uint32_t)(__ballot(kf) >> gbase) & ((1u << G) - 1u);
    if (!COUNT && kf) {
      const int32_t q = o + __popc(gm & ((1u << gi) - 1u));
      rowi[q] = jidx[e];
      cval[q] = m[e];
    }
    o += __popc(gm);
  }
  if (COUNT && valid && gi == 0) cnt[k] = o;
  if (COUNT) {
    // one atomic per wavefront
#pragma unroll
    for (int q = 32; q > 0; q >>= 1) nnear += __shfl_xor(nnear, q, 64);
    if (lane == 0 && nnear > 0) atomicAdd(nearc, (unsigned long long)nnear);
  }
}

template <class T>
void build_typed(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st, sai_precond_s* pc,
                 sai_build_stats* stats) {
  const Allocator& al = pc->al;
  const int32_t n = sp->n;
  EventTimer t_all, t_pat, t_ls, t_asm;
  t_all.start(st);
  t_pat.start(st);
  DBuf<int64_t> jptr, iptr;
  DBuf<int32_t> jidx, iidx, cntJ, cntI;
  const bool psai = o.pattern == SAI_PAT_PSAI_TOL;
  DBuf<double> m64, res64;  // PSAI(tol): values and residuals from the search
  int l_m = 0;
  if (o.pattern == SAI_PAT_SPAI)
    spai_patterns(sp, o, st, al, jptr, jidx, iptr, iidx, cntJ, cntI, &l_m);
  else if (psai)
    psai_patterns(sp, o, st, al, jptr, jidx, iptr, iidx, cntJ, cntI, m64, res64, &l_m);
  else
    build_patterns(sp, o.pattern, st, al, jptr, jidx, iptr, iidx, cntJ, cntI);
  t_pat.stop(st);
  int64_t tot[2];
  HIPC(hipMemcpyAsync(&tot[0], jptr.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(&tot[1], iptr.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  DBuf<int> mx(&al, 4);
  HIPC(hipMemsetAsync(mx.p, 0, 4 * sizeof(int), st));
  hipLaunchKernelGGL(k_stats, dim3(grid_for(n, NT, 256)), dim3(NT), 0, st, n, cntJ.p, cntI.p, nullptr, 0.0,
                     mx.p);
  LAUNCH_CHECK();
  int hmx[4];
  HIPC(hipMemcpyAsync(hmx, mx.p, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  const int64_t nnz_full = tot[0];

  t_ls.start(st);
  DBuf<T> mfull(&al, (size_t)nnz_full + 1);
  DBuf<double> res(&al, (size_t)n + 1);
  int64_t bcols[16] = {};
  int nsing = 0;
  if (psai) {
    // the search solved (and dropped) in float64; M takes the values in T
    hipLaunchKernelGGL((k_to_type<T>), dim3(grid_for(nnz_full, NT, 65536)), dim3(NT), 0, st, nnz_full,
                       m64.p, mfull.p);
    LAUNCH_CHECK();
    HIPC(hipMemcpyAsync(res.p, res64.p, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
  } else {
    nsing = solve_columns<T>(sp, jptr.p, jidx.p, iptr.p, iidx.p, cntJ.p, cntI.p, hmx[0], hmx[1],
                             mfull.p, res.p, bcols, al, st);
  }
  t_ls.stop(st);
  if (nsing > 0)
    SAI_THROW(SAI_ESINGULAR, "%d column least-squares blocks are rank deficient", nsing);

  t_asm.start(st);
  // PSAI(tol) dropped inside its loop: nothing more is dropped here
  const int drop = psai ? SAI_DROP_NONE : o.drop;
  double norm1 = 0.0;
  if (drop == SAI_DROP_TOLK) {
    DBuf<unsigned long long> nb(&al, 1);
    HIPC(hipMemsetAsync(nb.p, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_norm1, dim3(grid_for(n, NT)), dim3(NT), 0, st, n, sp->t_col_ptr.p,
                       sp->t_cval.p, nb.p);
    LAUNCH_CHECK();
    unsigned long long bits = read_scalar(nb.p, st);
    memcpy(&norm1, &bits, sizeof(double));
  }
  DBuf<int32_t> ccnt(&al, (size_t)n + 1);
  DBuf<unsigned long long> nearc(&al, 1);
  HIPC(hipMemsetAsync(nearc.p, 0, sizeof(unsigned long long), st));
  const double eta = sizeof(T) == 4 ? 1e-4 : 1e-12;
  const unsigned dgrid = grid_for((int64_t)n * 16, NT);
  hipLaunchKernelGGL((k_drop<T, true>), dim3(dgrid), dim3(NT), 0, st, n, jptr.p, jidx.p, mfull.p, drop,
                     o.tau, o.delta, norm1, ccnt.p, nullptr, nullptr, nullptr, eta, nearc.p);
  LAUNCH_CHECK();
  pc->col_ptr.alloc(&al, (size_t)n + 1);
  exclusive_scan_i32(ccnt.p, pc->col_ptr.p, n, al, st);
  const int32_t nnz = read_scalar(pc->col_ptr.p + n, st);
  pc->nnz = nnz;
  pc->row_idx.alloc(&al, (size_t)nnz + 1);
  pc->cval.alloc(&al, ((size_t)nnz + 1) * sizeof(T));
  hipLaunchKernelGGL((k_drop<T, false>), dim3(dgrid), dim3(NT), 0, st, n, jptr.p, jidx.p, mfull.p, drop,
                     o.tau, o.delta, norm1, nullptr, pc->col_ptr.p, pc->row_idx.p, (T*)pc->cval.p, eta,
                     nullptr);
  LAUNCH_CHECK();
  pc->row_ptr.alloc(&al, (size_t)n + 1);
  pc->col_idx.alloc(&al, (size_t)nnz + 1);
  pc->val.alloc(&al, ((size_t)nnz + 1) * sizeof(T));
  csr_transpose<T>(n, n, pc->col_ptr.p, pc->row_idx.p, (const T*)pc->cval.p, pc->row_ptr.p,
                   pc->col_idx.p, (T*)pc->val.p, al, st);
  t_asm.stop(st);
  t_all.stop(st);

  if (stats) {
    DBuf<int> so(&al, 4);
    HIPC(hipMemsetAsync(so.p, 0, 4 * sizeof(int), st));
    hipLaunchKernelGGL(k_stats, dim3(grid_for(n, NT, 256)), dim3(NT), 0, st, n, cntJ.p, cntI.p, res.p,
                       o.delta, so.p);
    LAUNCH_CHECK();
    int hs[4];
    HIPC(hipMemcpyAsync(hs, so.p, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    stats->n = n;
    stats->nnz_m = nnz;
    stats->nnz_m_full = nnz_full;
    stats->sum_i = tot[1];
    stats->max_i = hs[0];
    stats->max_j = hs[1];
    stats->n_c = hs[2];
    stats->spar = sp->nnz_t > 0 ? (double)nnz / (double)sp->nnz_t : 0.0;
    for (int v = 0; v < 16; ++v) stats->bucket_cols[v] = bcols[v];
    stats->t_pattern_ms = t_pat.ms();
    stats->t_ls_ms = t_ls.ms();
    stats->t_assemble_ms = t_asm.ms();
    stats->t_total_ms = t_all.ms();
    stats->s = sp->s;
    stats->p = sp->p;
    stats->l_m = l_m;
    stats->drop_flips = (int64_t)read_scalar(nearc.p, st);
  }
  if (o.keep_lists) {
    pc->j_ptr = std::move(jptr);
    pc->j_idx = std::move(jidx);
    pc->i_ptr = std::move(iptr);
    pc->i_idx = std::move(iidx);
    pc->res = std::move(res);
    DBuf<char> mf(&al, ((size_t)nnz_full + 1) * sizeof(T));
    HIPC(hipMemcpyAsync(mf.p, mfull.p, (size_t)nnz_full * sizeof(T), hipMemcpyDeviceToDevice, st));
    pc->m_full = std::move(mf);
  }
  HIPC(hipStreamSynchronize(st));
}

}  // namespace

void build_impl(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st, sai_precond_s* pc,
                sai_build_stats* stats) {
  if (o.pattern < SAI_PAT_A || o.pattern > SAI_PAT_PSAI_TOL) SAI_THROW(SAI_EINVAL, "bad pattern");
  if (o.drop < SAI_DROP_NONE || o.drop > SAI_DROP_TOLK) SAI_THROW(SAI_EINVAL, "bad drop mode");
  if (o.precision != SAI_FP32 && o.precision != SAI_FP64) SAI_THROW(SAI_EINVAL, "bad precision");
  pc->al = sp->al;
  pc->al.stream = st;
  pc->n = sp->n;
  pc->precision = o.precision;
  if (o.precision == SAI_FP32)
    build_typed<float>(sp, o, st, pc, stats);
  else
    build_typed<double>(sp, o, st, pc, stats);
}

}  // namespace sai
