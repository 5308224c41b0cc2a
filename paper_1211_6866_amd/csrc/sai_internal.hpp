// Internal declarations shared by the HIP translation units of libsai.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sai.h"

namespace sai {

// ------------------------------------------------------------------ errors --

struct Error {
  int code;
  std::string msg;
};

void set_last_error(const std::string& m);

#define SAI_THROW(code, ...)                                         \
  do {                                                               \
    char _b[512];                                                    \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                           \
    throw ::sai::Error{(code), std::string(_b)};                     \
  } while (0)

#define HIPC(call)                                                                  \
  do {                                                                              \
    hipError_t _e = (call);                                                         \
    if (_e != hipSuccess)                                                           \
      SAI_THROW(SAI_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),    \
                __FILE__, __LINE__);                                                \
  } while (0)

#define LAUNCH_CHECK() HIPC(hipGetLastError())

// --------------------------------------------------------------- allocation --

struct Allocator {
  sai_allocator a{nullptr, nullptr, nullptr};
  hipStream_t stream = nullptr;

  void* get(size_t bytes) const {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (a.alloc) {
      p = a.alloc(a.ctx, bytes, (void*)stream);
      if (!p) SAI_THROW(SAI_ENOMEM, "allocator returned NULL for %zu bytes", bytes);
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess || !p) SAI_THROW(SAI_ENOMEM, "hipMalloc(%zu) failed", bytes);
    }
    return p;
  }
  void put(void* p) const {
    if (!p) return;
    if (a.free)
      a.free(a.ctx, p, (void*)stream);
    else
      (void)hipFree(p);
  }
};

// Owning device buffer; freed through the allocator it came from.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  const Allocator* al = nullptr;
  DBuf() = default;
  DBuf(const Allocator* a, size_t count) { alloc(a, count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), al(o.al) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; al = o.al; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(const Allocator* a, size_t count) {
    release();
    al = a;
    n = count;
    p = static_cast<T*>(a->get(count * sizeof(T)));
  }
  void release() {
    if (p && al) al->put(p);
    p = nullptr;
    n = 0;
  }
  T* get() const { return p; }
};

// Pinned host staging for small readbacks.
struct HostStage {
  void* p = nullptr;
  size_t bytes = 0;
  explicit HostStage(size_t b) : bytes(b) { HIPC(hipHostMalloc(&p, b, hipHostMallocDefault)); }
  ~HostStage() { if (p) (void)hipHostFree(p); }
  template <class T> T* as() { return static_cast<T*>(p); }
};

// ------------------------------------------------------------------ handles --

}  // namespace sai

struct sai_split_s {
  sai::Allocator al;
  int32_t n = 0, s = 0, p = 0, keep = 0;
  int64_t nnz_a = 0, nnz_t = 0, nnz_u = 0;
  sai::DBuf<int32_t> t_row_ptr, t_col_idx, t_col_ptr, t_row_idx;
  sai::DBuf<double> t_val, t_cval;
  sai::DBuf<int32_t> dense_cols;
  sai::DBuf<int32_t> u_row_ptr, u_col;
  sai::DBuf<double> u_val;
  sai::DBuf<int32_t> a_row_ptr, a_col_idx;  // structure of A for gradients
  double norm1_t = 0.0;                       // ||A~||_1
};

struct sai_precond_s {
  sai::Allocator al;
  int32_t n = 0, precision = SAI_FP32;
  int64_t nnz = 0;
  sai::DBuf<int32_t> col_ptr, row_idx, row_ptr, col_idx;
  sai::DBuf<char> cval, val;  // float or double
  // optional inspection lists
  sai::DBuf<int64_t> j_ptr, i_ptr;
  sai::DBuf<int32_t> j_idx, i_idx;
  sai::DBuf<char> m_full;
  sai::DBuf<double> res;
};

namespace sai {

// -------------------------------------------------------- device utilities --

constexpr int WAVE = 64;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum over groups of G consecutive lanes (G a power of two <= 64).
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Block-wide sum for blockDim.x == NT (multiple of 64); result on every thread.
template <int NT, class T>
__device__ __forceinline__ T block_sum(T v, T* lds /* NT/64 */) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) lds[w] = v;
  __syncthreads();
  T t = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) t += lds[i];
  return t;
}

// Wave-aggregated counter increment: every lane with key >= 0 receives a slot
// in counter[key] (one atomicAdd per distinct key per wave instead of one per
// lane).  Must be called by all active lanes of the wave together.
__device__ __forceinline__ int agg_slot(int* counter, int key) {
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int slot = -1;
  unsigned long long pending = __ballot(key >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int lk = __shfl(key, leader, WAVE);
    const unsigned long long same = __ballot(key == lk);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counter[lk], __popcll(same));
    base = __shfl(base, leader, WAVE);
    if (key == lk) slot = base + __popcll(same & lt);
    pending &= ~same;
  }
  return slot;
}

// Block-aggregated slot allocation: every thread of the block calls it with a
// key in [0, NK) or -1; returns a distinct slot per key (global counter
// gcounter[key] advanced once per key per block; LDS atomics inside the
// block).  Order of the slots within a key is unspecified.
template <int NK>
__device__ __forceinline__ int block_slot(int* gcounter, int key) {
  __shared__ int lcnt[NK], lbase[NK];
  if (threadIdx.x < NK) lcnt[threadIdx.x] = 0;
  __syncthreads();
  const int local = key >= 0 ? atomicAdd(&lcnt[key], 1) : -1;
  __syncthreads();
  if (threadIdx.x < NK && lcnt[threadIdx.x] > 0) lbase[threadIdx.x] = atomicAdd(&gcounter[threadIdx.x], lcnt[threadIdx.x]);
  __syncthreads();
  const int slot = key >= 0 ? lbase[key] + local : -1;
  __syncthreads();
  return slot;
}

inline unsigned grid_for(int64_t work, int per_block, unsigned cap = 1u << 30) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (int64_t)cap) g = cap;
  return (unsigned)g;
}

// ------------------------------------------------------- host-side helpers --

// Exclusive prefix sum of n values into out[0..n]; out[n] = total.  `in` and
// `out` may alias only if in == out.  T = int32_t or int64_t.
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, const Allocator& al,
                        hipStream_t st);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, const Allocator& al,
                        hipStream_t st);
// Same with int32 input and int64 output.
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, const Allocator& al,
                               hipStream_t st);

template <class T>
T read_scalar(const T* dev, hipStream_t st) {
  T v;
  HIPC(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return v;
}

// Tuning knob `name` (kernel variant or size choice): the value of the
// environment variable SAI_TUNE_<name> if set, else `dflt`.
int tune_get(const char* name, int dflt);
void tune_set(const char* name, int value);
void tune_clear();

// Workgroups of `kernel` (nt threads, no dynamic LDS) resident on the current
// device at once (occupancy per CU times the CU count); cached per device.
int resident_blocks(const void* kernel, int nt);

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
void fill_f64(double* p, double v, int64_t n, hipStream_t st);
void zero_bytes(void* p, size_t bytes, hipStream_t st);

// Timing helper: events recorded on a stream.
struct EventTimer {
  hipEvent_t a = nullptr, b = nullptr;
  EventTimer() { HIPC(hipEventCreate(&a)); HIPC(hipEventCreate(&b)); }
  ~EventTimer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  void start(hipStream_t st) { HIPC(hipEventRecord(a, st)); }
  void stop(hipStream_t st) { HIPC(hipEventRecord(b, st)); }
  float ms() { HIPC(hipEventSynchronize(b)); float t = 0; HIPC(hipEventElapsedTime(&t, a, b)); return t; }
};

// ---------------------------------------------------------------- profiling --

// RAII scope: when profiling is enabled, records events around the launches
// made while it is alive, on stream `st`, under `name`.
struct ProfScope {
  int slot = -1;
  hipStream_t st = nullptr;
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
};
#define SAI_PROF(name, st) ::sai::ProfScope _sai_prof_scope_##__LINE__((name), (st))

// ------------------------------------------------------------ entry points --

void split_impl(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                const double* val, const sai_split_opts& o, const Allocator& al,
                sai_split_s* h);
void build_impl(const sai_split_s* sp, const sai_build_opts& o, hipStream_t st,
                sai_precond_s* pc, sai_build_stats* stats);
// Returns per-column iterations/status into host arrays (size k).
int krylov_impl(const sai_split_s* sp, const sai_precond_s* pc, int transpose, int k,
                const double* R, double* X, const double* thr, const sai_solve_opts& o,
                hipStream_t st, int32_t* iters, int32_t* status);
// SMW recovery x = y - W (I + V^T W)^{-1} V^T y on the device (LU in float64).
void smw_recover(const sai_split_s* sp, const double* Y, double* x, double* c_host,
                 hipStream_t st);
// smw_recover without any allocation: K, z and the pivot flag in the file-scope
// scratch array of smw.hip (s <= SMW_NOALLOC_SMAX).
constexpr int SMW_NOALLOC_SMAX = 64;
void smw_recover_noalloc(const sai_split_s* sp, const double* Y, double* x, double* c_host,
                         hipStream_t st);
// Standalone gather of the dense column blocks A~(I_k, J_k) (column-major, at
// blk_off[k] elements) in float (precision SAI_FP32) or double.
void gather_offsets(const sai_precond_s* pc, int64_t* blk_off, int64_t* total, hipStream_t st);
void gather_blocks(const sai_split_s* sp, const sai_precond_s* pc, int precision,
                   const int64_t* blk_off, void* blocks, hipStream_t st);
double residual_impl(const sai_split_s* sp, const double* b, const double* x, hipStream_t st);
void backward_impl(const sai_split_s* sp, const sai_precond_s* pc, const double* x,
                   const double* gx, double* gb, double* ga, const sai_solve_opts& o,
                   hipStream_t st, sai_solve_stats* stats);
// y_out (device, n x (s+1), may be null): receives the Krylov solutions [y, W]
void solve_impl(const sai_split_s* sp, const sai_precond_s* pc, const double* b, double* x,
                const sai_solve_opts& o, hipStream_t st, sai_solve_stats* stats, double* y_out = nullptr);
// the adjoint from the forward solve's W = Y[:, 1..s]: one system with A~^T per pass
void backward_y_impl(const sai_split_s* sp, const sai_precond_s* pc, const double* x, const double* Y,
                     const double* gx, double* gb, double* ga, const sai_solve_opts& o, hipStream_t st,
                     sai_solve_stats* stats);

// Device-wide deterministic float64 norms / dots (two-level, fixed order).
double dev_norm2(const double* v, int64_t n, int64_t stride, const Allocator& al, hipStream_t st);

// Dense s x s LU solve on the device (partial pivoting); K (row-major, s x s)
// and rhs (s) are overwritten; the solution is left in rhs.  nrhs columns in
// rhs (row-major s x nrhs).  Returns false if a zero pivot is met.
bool dense_lu_solve(double* K, double* rhs, int s, int nrhs, const Allocator& al, hipStream_t st);
// The same LU kernel on caller-provided memory; *fail (device) must be zero
// before the launch and is set on a zero pivot.  No allocation.
void launch_dense_lu(double* K, double* rhs, int s, int nrhs, int* fail, hipStream_t st);

}  // namespace sai
