// Device-wide scans, fills, deterministic norms and a small dense LU solver.
#include <algorithm>
#include <map>
#include <mutex>

#include "sai_internal.hpp"

namespace sai {

namespace {

constexpr int SCAN_NT = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_NT * SCAN_ITEMS;

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = threadIdx.x % WAVE;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T t = __shfl_up(v, o, WAVE);
    if (l >= o) v += t;
  }
  return v;
}

template <class TI, class TO>
__global__ void __launch_bounds__(SCAN_NT) k_scan_tile(const TI* in, TO* out, TO* tile_sum, int64_t n) {
  __shared__ TO wsum[SCAN_NT / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  TO v[SCAN_ITEMS];
  TO s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    v[i] = idx < n ? (TO)in[idx] : (TO)0;
    s += v[i];
  }
  TO incl = wave_incl_scan(s);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  if (l == WAVE - 1) wsum[w] = incl;
  __syncthreads();
  TO woff = 0;
  for (int i = 0; i < w; ++i) woff += wsum[i];
  incl += woff;
  TO ex = incl - s;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = ex;
    ex += v[i];
  }
  if (threadIdx.x == SCAN_NT - 1) tile_sum[blockIdx.x] = incl;
}

template <class TO>
__global__ void k_scan_add(TO* out, const TO* tile_off, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / SCAN_TILE];
}

template <class TO>
__global__ void k_set_total(TO* out, const TO* tile_sum_scanned, int64_t ntile, int64_t n) {
  // out[n] = exclusive offset of the last tile + its sum = scanned[ntile]
  out[n] = tile_sum_scanned[ntile];
}

template <class TI, class TO>
void scan_rec(const TI* in, TO* out, int64_t n, const Allocator& al, hipStream_t st) {
  const int64_t ntile = (n + SCAN_TILE - 1) / SCAN_TILE;
  DBuf<TO> ts(&al, ntile + 1);
  if (n > 0) {
    hipLaunchKernelGGL((k_scan_tile<TI, TO>), dim3((unsigned)ntile), dim3(SCAN_NT), 0, st, in, out,
                       ts.p, n);
    LAUNCH_CHECK();
  }
  if (ntile > 1) {
    scan_rec<TO, TO>(ts.p, ts.p, ntile, al, st);  // ts[0..ntile] exclusive, ts[ntile] = total
    hipLaunchKernelGGL((k_scan_add<TO>), dim3(grid_for(n, 256)), dim3(256), 0, st, out, ts.p, n);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_set_total<TO>), dim3(1), dim3(1), 0, st, out, ts.p, ntile, n);
    LAUNCH_CHECK();
  } else {
    // single tile: total = ts[0]
    if (n > 0) {
      HIPC(hipMemcpyAsync(out + n, ts.p, sizeof(TO), hipMemcpyDeviceToDevice, st));
    } else {
      HIPC(hipMemsetAsync(out, 0, sizeof(TO), st));
    }
  }
  // `ts` is released here; the allocator's reuse is ordered on `st` (torch's caching
  // allocator) or synchronising (hipFree), so pending kernels still see valid memory.
}

template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

constexpr int NORM_NT = 256;
constexpr int NORM_BLOCKS = 1024;

__global__ void __launch_bounds__(NORM_NT) k_sumsq_partial(const double* v, int64_t n, int64_t stride,
                                                           double* part) {
  __shared__ double lds[NORM_NT / WAVE];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * NORM_NT) {
    double t = v[i * stride];
    acc += t * t;
  }
  acc = block_sum<NORM_NT>(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(NORM_NT) k_sum_final(const double* part, int np, double* out) {
  __shared__ double lds[NORM_NT / WAVE];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += NORM_NT) acc += part[i];
  acc = block_sum<NORM_NT>(acc, lds);
  if (threadIdx.x == 0) out[0] = acc;
}

// One workgroup; K row-major s x s, rhs row-major s x nrhs.
constexpr int LU_NT = 256;
__global__ void __launch_bounds__(LU_NT) k_dense_lu(double* K, double* rhs, int s, int nrhs, int* fail) {
  __shared__ double bv[LU_NT];
  __shared__ int bi[LU_NT];
  __shared__ int piv_s;
  for (int j = 0; j < s; ++j) {
    // pivot: largest |K[i][j]|, i >= j, smallest i on ties
    double best = -1.0;
    int bidx = s;
    for (int i = j + threadIdx.x; i < s; i += LU_NT) {
      double a = fabs(K[(int64_t)i * s + j]);
      if (a > best) { best = a; bidx = i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = LU_NT / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        double a = bv[threadIdx.x + o];
        int ia = bi[threadIdx.x + o];
        if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ia < bi[threadIdx.x])) {
          bv[threadIdx.x] = a;
          bi[threadIdx.x] = ia;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) piv_s = bi[0];
    __syncthreads();
    const int piv = piv_s;
    if (!(bv[0] > 0.0)) {  // zero (or NaN) pivot
      if (threadIdx.x == 0) *fail = 1;
      return;
    }
    if (piv != j) {
      for (int c = threadIdx.x; c < s; c += LU_NT) {
        double t = K[(int64_t)j * s + c];
        K[(int64_t)j * s + c] = K[(int64_t)piv * s + c];
        K[(int64_t)piv * s + c] = t;
      }
      for (int c = threadIdx.x; c < nrhs; c += LU_NT) {
        double t = rhs[(int64_t)j * nrhs + c];
        rhs[(int64_t)j * nrhs + c] = rhs[(int64_t)piv * nrhs + c];
        rhs[(int64_t)piv * nrhs + c] = t;
      }
    }
    __syncthreads();
    const double d = K[(int64_t)j * s + j];
    // multipliers
    for (int i = j + 1 + threadIdx.x; i < s; i += LU_NT) K[(int64_t)i * s + j] /= d;
    __syncthreads();
    // trailing update of K and rhs
    const int rows = s - j - 1;
    const int wk = s - j - 1 + nrhs;
    for (int64_t t = threadIdx.x; t < (int64_t)rows * wk; t += LU_NT) {
      int i = j + 1 + (int)(t / wk);
      int c = (int)(t % wk);
      double l = K[(int64_t)i * s + j];
      if (c < s - j - 1) {
        int cc = j + 1 + c;
        K[(int64_t)i * s + cc] -= l * K[(int64_t)j * s + cc];
      } else {
        int cc = c - (s - j - 1);
        rhs[(int64_t)i * nrhs + cc] -= l * rhs[(int64_t)j * nrhs + cc];
      }
    }
    __syncthreads();
  }
  // back substitution, one thread per right-hand side column
  for (int c = threadIdx.x; c < nrhs; c += LU_NT) {
    for (int j = s - 1; j >= 0; --j) {
      double acc = rhs[(int64_t)j * nrhs + c];
      for (int q = j + 1; q < s; ++q) acc -= K[(int64_t)j * s + q] * rhs[(int64_t)q * nrhs + c];
      rhs[(int64_t)j * nrhs + c] = acc / K[(int64_t)j * s + j];
    }
  }
}

}  // namespace

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, const Allocator& al,
                        hipStream_t st) {
  scan_rec<int32_t, int32_t>(in, out, n, al, st);
}
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, const Allocator& al,
                        hipStream_t st) {
  scan_rec<int64_t, int64_t>(in, out, n, al, st);
}
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, const Allocator& al,
                               hipStream_t st) {
  scan_rec<int32_t, int64_t>(in, out, n, al, st);
}

// Launch-shape knobs: the environment (SAI_TUNE_<name>) wins, then the values
// set through sai_tune_set (a tuning file loaded by the caller), then the
// built-in default.
namespace {
std::mutex tune_mu;
std::map<std::string, int>& tune_table() {
  static std::map<std::string, int> t;
  return t;
}
}  // namespace

int tune_get(const char* name, int dflt) {
  char key[128];
  snprintf(key, sizeof(key), "SAI_TUNE_%s", name);
  const char* v = getenv(key);
  if (v && *v) return atoi(v);
  std::lock_guard<std::mutex> lk(tune_mu);
  auto it = tune_table().find(name);
  return it != tune_table().end() ? it->second : dflt;
}

void tune_set(const char* name, int value) {
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_table()[name] = value;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_table().clear();
}

int resident_blocks(const void* kernel, int nt) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({dev, kernel});
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0));
  const int r = std::max(1, cus * per_cu);
  cache[{dev, kernel}] = r;
  return r;
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_fill<int32_t>), dim3(grid_for(n, 256, 65536)), dim3(256), 0, st, p, v, n);
  LAUNCH_CHECK();
}
void fill_f64(double* p, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(n, 256, 65536)), dim3(256), 0, st, p, v, n);
  LAUNCH_CHECK();
}
void zero_bytes(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  HIPC(hipMemsetAsync(p, 0, bytes, st));
}

double dev_norm2(const double* v, int64_t n, int64_t stride, const Allocator& al, hipStream_t st) {
  DBuf<double> part(&al, NORM_BLOCKS + 1);
  unsigned nb = grid_for(n, NORM_NT, NORM_BLOCKS);
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nb), dim3(NORM_NT), 0, st, v, n, stride, part.p);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(NORM_NT), 0, st, part.p, (int)nb, part.p + NORM_BLOCKS);
  LAUNCH_CHECK();
  double r = read_scalar(part.p + NORM_BLOCKS, st);
  return std::sqrt(r);
}

void launch_dense_lu(double* K, double* rhs, int s, int nrhs, int* fail, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_lu, dim3(1), dim3(LU_NT), 0, st, K, rhs, s, nrhs, fail);
  LAUNCH_CHECK();
}

bool dense_lu_solve(double* K, double* rhs, int s, int nrhs, const Allocator& al, hipStream_t st) {
  if (s <= 0) return true;
  DBuf<int> fail(&al, 1);
  HIPC(hipMemsetAsync(fail.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_dense_lu, dim3(1), dim3(LU_NT), 0, st, K, rhs, s, nrhs, fail.p);
  LAUNCH_CHECK();
  return read_scalar(fail.p, st) == 0;
}

}  // namespace sai
