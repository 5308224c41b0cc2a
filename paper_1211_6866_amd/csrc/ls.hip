// Column least-squares solves: m_k = argmin ||A~(I_k, J_k) m - e_k(I_k)||
// (Section 2, (subprob) -> (lsprob)), by Householder QR and back-substitution.
//
// Register kernels (k_ls_qr): a group of G lanes (G = 16, 32 or 64) owns one
// problem; lane l of the group holds rows l, l+G, ..., l+(R-1)G of the dense
// block in registers, so the factorisation never touches memory.  Column
// reductions are butterfly sums over the group: four DPP steps inside a row of
// 16 lanes (quad_perm xor-1, quad_perm xor-2, row_half_mirror, row_mirror),
// plus cross-row shuffles for G = 32/64.  Every lane of a group receives the
// bit-identical sum.  The j (reflector) and c (column) loops are fully
// unrolled so that all register indices are static; a wave-uniform guard
// skips the steps past the widest problem of the wave.
//
// The block is gathered first, one problem at a time, through an LDS tile: the
// entries of the columns A~(:, j), j in J_k, are scattered to the position of
// their row in I_k (binary search in the sorted I_k).
//
// Large problems (k_ls_qr_big) use one 256-thread workgroup with the block in a
// global workspace.
#include "sai_internal.hpp"

#include <algorithm>

namespace sai {

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the G consecutive lanes of a group; identical result in every lane.
template <int G, class T>
__device__ __forceinline__ T gsum(T v) {
  static_assert(G == 16 || G == 32 || G == 64, "group size");
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// gsum over N independent values at once: the DPP steps of the N sums are
// interleaved, so no step waits on the one just before it (each value gets the
// same sequence of additions as gsum).  Only the first cnt values are summed
// (cnt is a constant once the caller's loops are unrolled).
template <int G, int N, class T>
__device__ __forceinline__ void gsum_n(T (&v)[N], int cnt) {
  static_assert(G == 16 || G == 32 || G == 64, "group size");
#pragma unroll
  for (int u = 0; u < N; ++u) if (u < cnt) v[u] += dpp_mov<0xB1>(v[u]);
#pragma unroll
  for (int u = 0; u < N; ++u) if (u < cnt) v[u] += dpp_mov<0x4E>(v[u]);
#pragma unroll
  for (int u = 0; u < N; ++u) if (u < cnt) v[u] += dpp_mov<0x141>(v[u]);
#pragma unroll
  for (int u = 0; u < N; ++u) if (u < cnt) v[u] += dpp_mov<0x140>(v[u]);
  if constexpr (G >= 32) {
#pragma unroll
    for (int u = 0; u < N; ++u) if (u < cnt) v[u] += __shfl_xor(v[u], 16, 64);
  }
  if constexpr (G >= 64) {
#pragma unroll
    for (int u = 0; u < N; ++u) if (u < cnt) v[u] += __shfl_xor(v[u], 32, 64);
  }
}

// Value of lane src (0 <= src < G) of the caller's group, in every lane of the
// group.  G = 16: one DPP row broadcast (row_newbcast); src must be a constant
// once the caller's loops are unrolled.
template <int G, class T>
__device__ __forceinline__ T gbcast(T v, int src) {
  if constexpr (G == 16) {
    switch (src) {
      case 0: return dpp_mov<0x150>(v);
      case 1: return dpp_mov<0x151>(v);
      case 2: return dpp_mov<0x152>(v);
      case 3: return dpp_mov<0x153>(v);
      case 4: return dpp_mov<0x154>(v);
      case 5: return dpp_mov<0x155>(v);
      case 6: return dpp_mov<0x156>(v);
      case 7: return dpp_mov<0x157>(v);
      case 8: return dpp_mov<0x158>(v);
      case 9: return dpp_mov<0x159>(v);
      case 10: return dpp_mov<0x15A>(v);
      case 11: return dpp_mov<0x15B>(v);
      case 12: return dpp_mov<0x15C>(v);
      case 13: return dpp_mov<0x15D>(v);
      case 14: return dpp_mov<0x15E>(v);
      default: return dpp_mov<0x15F>(v);
    }
  } else {
    return __shfl(v, (int)(threadIdx.x & (64 - G)) + src, 64);
  }
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int lower_bound_lds(const int32_t* a, int n, int32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <class T, int G, int R, int JMAX, int MINW = 1>
__global__ void __launch_bounds__(64, MINW) k_ls_qr(const int32_t* __restrict__ cols, int ncols,
                                              const int64_t* __restrict__ jptr,
                                              const int32_t* __restrict__ jidx,
                                              const int64_t* __restrict__ iptr,
                                              const int32_t* __restrict__ iidx,
                                              const int32_t* __restrict__ cp,
                                              const int32_t* __restrict__ ri,
                                              const double* __restrict__ cv, T* __restrict__ mout,
                                              double* __restrict__ res_out, int* __restrict__ nsing) {
  constexpr int NP = 64 / G;
  constexpr int ROWS = G * R;
  constexpr int LDT = JMAX + 1;
  constexpr int MS = (JMAX + G - 1) / G;
  // columns reflected together (interleaved group sums); wider groups keep the
  // larger variants from being fully unrolled, which would put a[][] in scratch
  constexpr int GW = (G == 16 && sizeof(T) == 4) ? 4 : 1;
  static_assert(JMAX <= ROWS, "row slots must cover the columns");
  __shared__ T tile[ROWS * LDT];
  __shared__ int32_t sI[ROWS];
  __shared__ int32_t sStart[JMAX];
  __shared__ int32_t sOff[JMAX + 1];

  const int lane = threadIdx.x;
  const int g = lane / G;
  const int li = lane % G;

  for (int64_t base = (int64_t)blockIdx.x * NP; base < ncols; base += (int64_t)gridDim.x * NP) {
    const int64_t myidx = base + g;
    const bool valid = myidx < ncols;
    const int k = valid ? cols[myidx] : -1;
    const int nJ = valid ? (int)(jptr[k + 1] - jptr[k]) : 0;
    const int nI = valid ? (int)(iptr[k + 1] - iptr[k]) : 0;

    T a[R][JMAX];
    T b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      b[r] = 0;
#pragma unroll
      for (int c = 0; c < JMAX; ++c) a[r][c] = 0;
    }

    // ---- gather, one problem of the wave at a time
    for (int p = 0; p < NP; ++p) {
      const int kp = __shfl(k, p * G, 64);
      if (kp < 0) continue;
      const int nJp = __shfl(nJ, p * G, 64);
      const int nIp = __shfl(nI, p * G, 64);
      const int64_t jo = jptr[kp], io = iptr[kp];
      int cnt = 0;
      if (lane < nJp) {
        const int32_t j = jidx[jo + lane];
        const int32_t s0 = cp[j];
        cnt = cp[j + 1] - s0;
        sStart[lane] = s0;
      }
      int incl = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane < nJp) sOff[lane] = incl - cnt;
      const int total = __shfl(incl, 63, 64);
      if (lane == 0) sOff[nJp] = total;
      for (int t = lane; t < nIp; t += 64) sI[t] = iidx[io + t];
      for (int t = lane; t < ROWS * LDT; t += 64) tile[t] = (T)0;
      __syncthreads();
      for (int f = lane; f < total; f += 64) {
        int lo = 0, hi = nJp - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (sOff[mid] <= f) lo = mid; else hi = mid - 1;
        }
        const int32_t e = sStart[lo] + (f - sOff[lo]);
        const int pos = lower_bound_lds(sI, nIp, ri[e]);
        tile[pos * LDT + lo] = (T)cv[e];
      }
      __syncthreads();
      if (g == p) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rho = li + G * r;
          if (rho < nIp) {
#pragma unroll
            for (int c = 0; c < JMAX; ++c) a[r][c] = tile[rho * LDT + c];
            b[r] = (sI[rho] == kp) ? (T)1 : (T)0;
          }
        }
      }
      __syncthreads();
    }

    // wave-uniform (a scalar), so that the guards below are scalar branches
    const int nJmax = __builtin_amdgcn_readfirstlane(wave_max_i(nJ));
    bool sing = false;

    // ---- Householder QR; Q^T is applied to the right-hand side as we go
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      if (j < nJmax) {
        const bool act = j < nJ;
        T tail = 0, ap = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rho = li + G * r;
          const T x = a[r][j];
          if (rho > j) tail += x * x;
          if (rho == j) ap = x;
        }
        T ta[2] = {tail, ap};
        gsum_n<G>(ta, 2);
        tail = ta[0];
        const T alpha = ta[1];
        const T normx = sqrt(tail + alpha * alpha);
        const T sgn = alpha >= (T)0 ? (T)1 : (T)-1;
        const T vj = alpha + sgn * normx;
        const T vtv = tail + vj * vj;
        const bool ok = act && normx > (T)0;
        if (act && !(normx > (T)0)) sing = true;
        const T tau = ok ? (T)2 / vtv : (T)0;
        T v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rho = li + G * r;
          v[r] = rho > j ? a[r][j] : (rho == j ? vj : (T)0);
        }
        // reflect the right-hand side and columns j+1 .. JMAX-1, GW at a time
        // (first group: b and columns j+1 .. j+GW-1), their group sums
        // interleaved
        {
          T d[GW];
          d[0] = 0;
#pragma unroll
          for (int r = 0; r < R; ++r) d[0] += v[r] * b[r];
#pragma unroll
          for (int u = 1; u < GW; ++u) {
            d[u] = 0;
            if (j + u < JMAX) {
#pragma unroll
              for (int r = 0; r < R; ++r) d[u] += v[r] * a[r][j + u];
            }
          }
          const int cnt = JMAX - j < GW ? JMAX - j : GW;
          gsum_n<G>(d, cnt);
#pragma unroll
          for (int r = 0; r < R; ++r) b[r] -= (tau * d[0]) * v[r];
#pragma unroll
          for (int u = 1; u < GW; ++u) {
            if (j + u < JMAX) {
              const T f = tau * d[u];
#pragma unroll
              for (int r = 0; r < R; ++r) a[r][j + u] -= f * v[r];
            }
          }
        }
#pragma unroll
        for (int c0 = j + GW; c0 < JMAX; c0 += GW) {
          if (c0 < nJmax) {
            T d[GW];
#pragma unroll
            for (int u = 0; u < GW; ++u) {
              d[u] = 0;
              if (c0 + u < JMAX) {
#pragma unroll
                for (int r = 0; r < R; ++r) d[u] += v[r] * a[r][c0 + u];
              }
            }
            const int cnt = JMAX - c0 < GW ? JMAX - c0 : GW;
            gsum_n<G>(d, cnt);
#pragma unroll
            for (int u = 0; u < GW; ++u) {
              if (c0 + u < JMAX) {
                const T f = tau * d[u];
#pragma unroll
                for (int r = 0; r < R; ++r) a[r][c0 + u] -= f * v[r];
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rho = li + G * r;
          if (rho == j && act) a[r][j] = -sgn * normx;
        }
      }
    }

    // ---- back-substitution R m = (Q^T e)[0:nJ]
    T macc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) macc[r] = 0;
    T mown[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) mown[q] = 0;
#pragma unroll
    for (int c = JMAX - 1; c >= 0; --c) {
      if (c < nJmax) {
        const int rc = c / G;
        T part = 0;
        if (c < nJ && li == c % G && !sing) part = (b[rc] - macc[rc]) / a[rc][c];
        const T mc = gbcast<G>(part, c % G);
        if (li == c % G) mown[c / G] = mc;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rho = li + G * r;
          if (rho < c) macc[r] += a[r][c] * mc;
        }
      }
    }
    T rs = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int rho = li + G * r;
      if (rho >= nJ) rs += b[r] * b[r];
    }
    rs = gsum<G>(rs);
    if (valid) {
      const int64_t jo = jptr[k];
#pragma unroll
      for (int q = 0; q < MS; ++q) {
        const int c = li + G * q;
        if (c < nJ) mout[jo + c] = mown[q];
      }
      if (li == 0) {
        res_out[k] = (double)sqrt(rs);
        if (sing) atomicAdd(nsing, 1);
      }
    }
  }
}

// ---- large problems: one workgroup, block in global memory ------------------

constexpr int BIG_NT = 1024;  // 16 wavefronts: the column updates of a step spread over them
constexpr int BIG_MAXI = 8192;  // the large search limits of spai.hip (CapL)
constexpr int BIG_MAXJ = 512;

template <class T>
__global__ void __launch_bounds__(BIG_NT) k_ls_qr_big(const int32_t* __restrict__ cols, int ncols,
                                                      const int64_t* __restrict__ jptr,
                                                      const int32_t* __restrict__ jidx,
                                                      const int64_t* __restrict__ iptr,
                                                      const int32_t* __restrict__ iidx,
                                                      const int32_t* __restrict__ cp,
                                                      const int32_t* __restrict__ ri,
                                                      const double* __restrict__ cv,
                                                      T* __restrict__ work, int64_t work_stride,
                                                      T* __restrict__ mout, double* __restrict__ res_out,
                                                      int* __restrict__ nsing, int* __restrict__ next) {
  __shared__ int32_t sI[BIG_MAXI];
  __shared__ int32_t sStart[BIG_MAXJ];
  __shared__ int32_t sOff[BIG_MAXJ + 1];
  __shared__ T sd[BIG_MAXJ + 1];
  __shared__ T sm[BIG_MAXJ];
  __shared__ T red[BIG_NT / 64];
  __shared__ T s_tail[2];
  __shared__ int s_q;
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  T* W = work + (int64_t)blockIdx.x * work_stride;
  // problems are taken one at a time from the counter `next` (the list holds
  // the costliest first), so that no workgroup is left with a queue of them
  for (;;) {
    __syncthreads();  // every thread has read the previous s_q
    if (tid == 0) s_q = atomicAdd(next, 1);
    __syncthreads();
    const int q = s_q;
    if (q >= ncols) break;
    const int k = cols[q];
    const int64_t jo = jptr[k], io = iptr[k];
    const int nJ = (int)(jptr[k + 1] - jo), nI = (int)(iptr[k + 1] - io);
    T* bvec = W + (int64_t)nI * nJ;  // column nJ of the workspace = right-hand side
    for (int t = tid; t < nI; t += BIG_NT) sI[t] = iidx[io + t];
    if (tid == 0) {
      int acc = 0;
      for (int c = 0; c < nJ; ++c) {
        const int32_t j = jidx[jo + c];
        sStart[c] = cp[j];
        sOff[c] = acc;
        acc += cp[j + 1] - cp[j];
      }
      sOff[nJ] = acc;
    }
    for (int64_t t = tid; t < (int64_t)nI * (nJ + 1); t += BIG_NT) W[t] = (T)0;
    __syncthreads();
    const int total = sOff[nJ];
    for (int f = tid; f < total; f += BIG_NT) {
      int lo = 0, hi = nJ - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sOff[mid] <= f) lo = mid; else hi = mid - 1;
      }
      const int32_t e = sStart[lo] + (f - sOff[lo]);
      const int pos = lower_bound_lds(sI, nI, ri[e]);
      W[(int64_t)lo * nI + pos] = (T)cv[e];
    }
    for (int t = tid; t < nI; t += BIG_NT) bvec[t] = (sI[t] == k) ? (T)1 : (T)0;
    __syncthreads();
    // Householder steps.  Column c (c = nJ: the right-hand side) belongs to
    // wavefront c % NW and its storage row t to lane t % 64, so a column's dot
    // with the reflector and its update need no barrier; the owner of the next
    // pivot column also sums that column's tail, and one barrier ends a step.
    // Row j of pivot column j is not read after step j starts (the reflector's
    // leading entry is vj, held by every thread), so R_jj is written by its
    // owner lane at the next step.
    constexpr int NW = BIG_NT / 64;
    bool sing = false;
    if (w == 0) {
      T tl = 0;
      for (int t = 1 + lane; t < nI; t += 64) tl += W[t] * W[t];
      tl = wave_sum(tl);
      if (lane == 0) s_tail[0] = tl;
    }
    __syncthreads();
    int jprev = -1;
    T rprev = 0;
    for (int j = 0; j < nJ; ++j) {
      if (jprev >= 0 && jprev < nI && w == jprev % NW && lane == jprev % 64)
        W[(int64_t)jprev * nI + jprev] = rprev;
      const T* colj = W + (int64_t)j * nI;
      const T tail = s_tail[j & 1];
      const T alpha = j < nI ? colj[j] : (T)0;
      const T normx = sqrt(tail + alpha * alpha);
      const T sgn = alpha >= (T)0 ? (T)1 : (T)-1;
      const T vj = alpha + sgn * normx;
      const T vtv = tail + vj * vj;
      const bool ok = normx > (T)0;
      if (!ok) sing = true;
      const T tau = ok ? (T)2 / vtv : (T)0;
      for (int c = j + 1 + ((w - (j + 1) % NW) + NW) % NW; c <= nJ; c += NW) {
        T* colc = W + (int64_t)c * nI;
        T d = 0;
        for (int t = j + lane; t < nI; t += 64) d += (t == j ? vj : colj[t]) * colc[t];
        d = tau * wave_sum(d);
        T nt = 0;
        for (int t = j + lane; t < nI; t += 64) {
          const T u = colc[t] - d * (t == j ? vj : colj[t]);
          colc[t] = u;
          if (t > j + 1) nt += u * u;
        }
        if (c == j + 1) {
          nt = wave_sum(nt);
          if (lane == 0) s_tail[(j + 1) & 1] = nt;
        }
      }
      jprev = j;
      rprev = -sgn * normx;
      __syncthreads();
    }
    if (jprev >= 0 && jprev < nI && w == jprev % NW && lane == jprev % 64)
      W[(int64_t)jprev * nI + jprev] = rprev;
    __syncthreads();
    // back-substitution (one wave)
    if (w == 0) {
      for (int c = nJ - 1; c >= 0; --c) {
        T part = 0;
        for (int q2 = c + 1 + lane; q2 < nJ; q2 += 64) part += W[(int64_t)q2 * nI + c] * sm[q2];
        part = wave_sum(part);
        if (lane == 0) sm[c] = sing ? (T)0 : (bvec[c] - part) / W[(int64_t)c * nI + c];
        // sm is written and read by this wave only; LDS accesses of one wave are in order
      }
    }
    __syncthreads();
    T rs = 0;
    for (int t = nJ + tid; t < nI; t += BIG_NT) rs += bvec[t] * bvec[t];
    rs = block_sum<BIG_NT>(rs, red);
    __syncthreads();
    for (int c = tid; c < nJ; c += BIG_NT) mout[jo + c] = sm[c];
    if (tid == 0) {
      res_out[k] = (double)sqrt(rs);
      if (sing) atomicAdd(nsing, 1);
    }
    __syncthreads();
  }
}

// ---- bucketing and dispatch ---------------------------------------------------

struct Variant {
  int maxI, maxJ;
};

template <class T>
struct VariantTable;

// float: register variants, then the global-memory kernel
template <>
struct VariantTable<float> {
  static constexpr int N = 8;
  static constexpr Variant v[N] = {{16, 8}, {32, 16}, {64, 25}, {64, 32}, {128, 32}, {256, 32},
                                   {128, 64}, {BIG_MAXI, BIG_MAXJ}};
};
template <>
struct VariantTable<double> {
  static constexpr int N = 9;
  static constexpr Variant v[N] = {{16, 8}, {32, 16}, {64, 25}, {64, 32}, {128, 32}, {256, 16},
                                   {256, 32}, {64, 64}, {BIG_MAXI, BIG_MAXJ}};
};

constexpr int BK_NT = 1024;
constexpr int BK_MAXV = 16;  // variants + 1 (the "too big" key)

__global__ void __launch_bounds__(BK_NT) k_bucket_assign(int32_t n, const int32_t* __restrict__ cntJ,
                                                         const int32_t* __restrict__ cntI, int nv,
                                                         const int* __restrict__ vmaxI,
                                                         const int* __restrict__ vmaxJ,
                                                         int32_t* __restrict__ bucket,
                                                         int* __restrict__ bcount) {
  __shared__ int lcnt[BK_MAXV];
  if (threadIdx.x < BK_MAXV) lcnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t k = (int64_t)blockIdx.x * BK_NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * BK_NT) {
    int b = -1;
    for (int v = 0; v < nv; ++v)
      if (cntI[k] <= vmaxI[v] && cntJ[k] <= vmaxJ[v]) { b = v; break; }
    bucket[k] = b;
    atomicAdd(&lcnt[b < 0 ? nv : b], 1);
  }
  __syncthreads();
  if ((int)threadIdx.x <= nv && lcnt[threadIdx.x] > 0) atomicAdd(&bcount[threadIdx.x], lcnt[threadIdx.x]);
}

__global__ void __launch_bounds__(BK_NT) k_bucket_scatter(int32_t n, const int32_t* __restrict__ bucket,
                                                          const int64_t* __restrict__ boff,
                                                          int* __restrict__ bcur,
                                                          int32_t* __restrict__ lists) {
  // every thread of the block runs the same number of iterations (block_slot syncs)
  for (int64_t k0 = (int64_t)blockIdx.x * BK_NT; k0 < n; k0 += (int64_t)gridDim.x * BK_NT) {
    const int64_t k = k0 + threadIdx.x;
    const int b = k < n ? bucket[k] : -1;
    const int slot = block_slot<BK_MAXV>(bcur, b);
    if (b >= 0) lists[boff[b] + slot] = (int32_t)k;
  }
}

// Work of each listed problem, |I| |J|^2 (the Householder flops up to a constant).
__global__ void __launch_bounds__(256) k_qr_cost(int cnt, const int32_t* __restrict__ list,
                                                 const int64_t* __restrict__ jptr,
                                                 const int64_t* __restrict__ iptr, int64_t* __restrict__ cost) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= cnt) return;
  const int k = list[t];
  const int64_t nJ = jptr[k + 1] - jptr[k], nI = iptr[k + 1] - iptr[k];
  cost[t] = nI * nJ * nJ;
}

// Reorder list[0..cnt) by decreasing cost (stable), for the global-memory kernel.
void order_by_cost(int32_t* list, int cnt, const int64_t* jptr, const int64_t* iptr, const Allocator& al,
                   hipStream_t st) {
  DBuf<int64_t> cost(&al, (size_t)cnt);
  hipLaunchKernelGGL(k_qr_cost, dim3(grid_for(cnt, 256)), dim3(256), 0, st, cnt, list, jptr, iptr, cost.p);
  LAUNCH_CHECK();
  std::vector<int32_t> hl((size_t)cnt), sl((size_t)cnt);
  std::vector<int64_t> hc((size_t)cnt);
  std::vector<int> ord((size_t)cnt);
  HIPC(hipMemcpyAsync(hl.data(), list, sizeof(int32_t) * (size_t)cnt, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(hc.data(), cost.p, sizeof(int64_t) * (size_t)cnt, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  for (int i = 0; i < cnt; ++i) ord[(size_t)i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return hc[(size_t)a] > hc[(size_t)b]; });
  for (int i = 0; i < cnt; ++i) sl[(size_t)i] = hl[(size_t)ord[(size_t)i]];
  HIPC(hipMemcpyAsync(list, sl.data(), sizeof(int32_t) * (size_t)cnt, hipMemcpyHostToDevice, st));
  HIPC(hipStreamSynchronize(st));
}

template <class T, int G, int R, int JMAX, int MINW = 1>
void launch_qr(const int32_t* list, int cnt, const int64_t* jptr, const int32_t* jidx,
               const int64_t* iptr, const int32_t* iidx, const sai_split_s* sp, T* mout,
               double* res, int* nsing, hipStream_t st) {
  if (cnt <= 0) return;
  constexpr int NP = 64 / G;
  const unsigned grid = grid_for(cnt, NP, 1u << 20);
  static char name[64];
  if (!name[0])
    snprintf(name, sizeof(name), "ls_qr_%s_g%dr%dj%d", sizeof(T) == 4 ? "f32" : "f64", G, R, JMAX);
  SAI_PROF(name, st);
  hipLaunchKernelGGL((k_ls_qr<T, G, R, JMAX, MINW>), dim3(grid), dim3(64), 0, st, list, cnt, jptr, jidx,
                     iptr, iidx, sp->t_col_ptr.p, sp->t_row_idx.p, sp->t_cval.p, mout, res, nsing);
  LAUNCH_CHECK();
}

template <class T>
void dispatch_variant(int v, const int32_t* list, int cnt, const int64_t* jptr,
                      const int32_t* jidx, const int64_t* iptr, const int32_t* iidx,
                      const sai_split_s* sp, T* mout, double* res, int* nsing, int maxI, int maxJ,
                      const Allocator& al, hipStream_t st) {
  if (cnt <= 0) return;
  constexpr bool F = sizeof(T) == 4;
  if constexpr (F) {
    switch (v) {
      case 0: launch_qr<T, 16, 1, 8>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 1: launch_qr<T, 16, 2, 16>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 2:  // 25-column problems (interior columns of P(|A~|^2) on 3D 7-point grids),
               // held to 168 registers so that three wavefronts share a SIMD
        launch_qr<T, 16, 4, 25, 3>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st);
        return;
      case 3: launch_qr<T, 16, 4, 32>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 4: launch_qr<T, 64, 2, 32>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 5: launch_qr<T, 64, 4, 32>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 6: launch_qr<T, 64, 2, 64>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      default: break;
    }
  } else {
    switch (v) {
      case 0: launch_qr<T, 16, 1, 8>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 1: launch_qr<T, 16, 2, 16>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 2: launch_qr<T, 16, 4, 25>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 3: launch_qr<T, 32, 2, 32>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 4: launch_qr<T, 64, 2, 32>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 5: launch_qr<T, 64, 4, 16>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 6: launch_qr<T, 64, 4, 32>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      case 7: launch_qr<T, 64, 1, 64>(list, cnt, jptr, jidx, iptr, iidx, sp, mout, res, nsing, st); return;
      default: break;
    }
  }
  // global-memory kernel for everything larger: one block (|I| x (|J| + 1))
  // per workgroup, at most 4 GB of them (problems come from a queue)
  const int64_t stride = (int64_t)maxI * (maxJ + 1);
  const int64_t wmax = std::max<int64_t>(1, (int64_t(4) << 30) / (stride * (int64_t)sizeof(T)));
  const unsigned grid = (unsigned)std::min<int64_t>({(int64_t)cnt, 1024, wmax});
  DBuf<T> work(&al, (size_t)grid * stride);
  DBuf<int> next(&al, 1);
  HIPC(hipMemsetAsync(next.p, 0, sizeof(int), st));
  SAI_PROF(sizeof(T) == 4 ? "ls_qr_f32_big" : "ls_qr_f64_big", st);
  hipLaunchKernelGGL((k_ls_qr_big<T>), dim3(grid), dim3(BIG_NT), 0, st, list, cnt, jptr, jidx, iptr,
                     iidx, sp->t_col_ptr.p, sp->t_row_idx.p, sp->t_cval.p, work.p, stride, mout, res,
                     nsing, next.p);
  LAUNCH_CHECK();
  HIPC(hipStreamSynchronize(st));
}

// Solve every column's LS problem; mout is indexed like jidx.  Returns the
// number of columns whose block was rank deficient.  bucket_cols (host, 16) gets
// the number of columns per kernel variant.
template <class T>
int solve_columns(const sai_split_s* sp, const int64_t* jptr, const int32_t* jidx,
                  const int64_t* iptr, const int32_t* iidx, const int32_t* cntJ,
                  const int32_t* cntI, int maxI, int maxJ, T* mout, double* res,
                  int64_t* bucket_cols, const Allocator& al, hipStream_t st) {
  using VT = VariantTable<T>;
  const int32_t n = sp->n;
  constexpr int NV = VT::N;
  // bucket edges: a column goes to the first variant v with |I| <= edgeI[v] and
  // |J| <= edgeJ[v]; the edges default to the variants' capacities and can be
  // lowered (0 disables a variant) by the knobs LSB_<F32|F64>_<v>_I / _J, which
  // the autotuner sets per workload class.  The last variant (global memory)
  // always keeps its capacity, so every column within the limits has a home.
  int hmaxI[NV], hmaxJ[NV];
  for (int v = 0; v < NV; ++v) {
    hmaxI[v] = VT::v[v].maxI;
    hmaxJ[v] = VT::v[v].maxJ;
    if (v < NV - 1) {
      char kn[64];
      snprintf(kn, sizeof(kn), "LSB_%s_%d_I", sizeof(T) == 4 ? "F32" : "F64", v);
      hmaxI[v] = std::max(0, std::min(hmaxI[v], tune_get(kn, hmaxI[v])));
      snprintf(kn, sizeof(kn), "LSB_%s_%d_J", sizeof(T) == 4 ? "F32" : "F64", v);
      hmaxJ[v] = std::max(0, std::min(hmaxJ[v], tune_get(kn, hmaxJ[v])));
    }
  }
  DBuf<int> vmax(&al, 2 * NV), bcount(&al, NV + 1), bcur(&al, NV + 1), nsing(&al, 1);
  DBuf<int32_t> bucket(&al, (size_t)n);
  HIPC(hipMemcpyAsync(vmax.p, hmaxI, sizeof(int) * NV, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(vmax.p + NV, hmaxJ, sizeof(int) * NV, hipMemcpyHostToDevice, st));
  HIPC(hipMemsetAsync(bcount.p, 0, sizeof(int) * (NV + 1), st));
  HIPC(hipMemsetAsync(bcur.p, 0, sizeof(int) * (NV + 1), st));
  HIPC(hipMemsetAsync(nsing.p, 0, sizeof(int), st));
  static_assert(NV + 1 <= BK_MAXV, "bucket keys");
  static_assert(NV <= 16, "bucket_cols holds 16 variants");
  hipLaunchKernelGGL(k_bucket_assign, dim3(grid_for(n, BK_NT, 512)), dim3(BK_NT), 0, st, n, cntJ, cntI, NV,
                     vmax.p, vmax.p + NV, bucket.p, bcount.p);
  LAUNCH_CHECK();
  int hc[NV + 1];
  HIPC(hipMemcpyAsync(hc, bcount.p, sizeof(int) * (NV + 1), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (hc[NV] > 0)
    SAI_THROW(SAI_ETOOBIG, "%d columns exceed |I| <= %d or |J| <= %d", hc[NV], BIG_MAXI, BIG_MAXJ);
  int64_t hoff[NV + 1];
  hoff[0] = 0;
  for (int v = 0; v < NV; ++v) hoff[v + 1] = hoff[v] + hc[v];
  DBuf<int64_t> boff(&al, NV + 1);
  DBuf<int32_t> lists(&al, (size_t)n + 1);
  HIPC(hipMemcpyAsync(boff.p, hoff, sizeof(int64_t) * (NV + 1), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_bucket_scatter, dim3(grid_for(n, BK_NT, 512)), dim3(BK_NT), 0, st, n, bucket.p,
                     boff.p, bcur.p, lists.p);
  LAUNCH_CHECK();
  for (int v = 0; v < NV; ++v) {
    if (bucket_cols) bucket_cols[v] = hc[v];
    // the order matters only when there are more problems than resident workgroups
    if (v == NV - 1 && hc[v] > std::min(1024, resident_blocks((const void*)k_ls_qr_big<T>, BIG_NT)))
      order_by_cost(lists.p + hoff[v], hc[v], jptr, iptr, al, st);
    dispatch_variant<T>(v, lists.p + hoff[v], hc[v], jptr, jidx, iptr, iidx, sp, mout, res, nsing.p,
                        maxI, maxJ, al, st);
  }
  return read_scalar(nsing.p, st);
}

template int solve_columns<float>(const sai_split_s*, const int64_t*, const int32_t*, const int64_t*,
                                  const int32_t*, const int32_t*, const int32_t*, int, int, float*,
                                  double*, int64_t*, const Allocator&, hipStream_t);
template int solve_columns<double>(const sai_split_s*, const int64_t*, const int32_t*, const int64_t*,
                                   const int32_t*, const int32_t*, const int32_t*, int, int, double*,
                                   double*, int64_t*, const Allocator&, hipStream_t);

}  // namespace sai
