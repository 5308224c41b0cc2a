// SMW recovery, residual check, Procedure * end to end, and the adjoint.
//
// Recovery (Procedure * step 3, (update1); Section 4 (composi)): with
// Y = [y_hat, W_hat] (n x (s+1), row-major) and V = (e_{j_1} .. e_{j_s}),
//   K = I + W_hat(j_d, :),  z = K^{-1} y_hat(j_d),  x = y_hat - W_hat z,
// K factored by LU with partial pivoting in float64; c = ||z||.
// Residual (rrnorm): rr = ||b - A~ x - U x(j)|| / ||b||, A = A~ + U V^T.
// Adjoint (Theorem 3.1 applied to A^T = A~^T + V U^T): A~^T [eta, Z] =
// [g, V], K' = I + U^T Z, lambda = eta - Z K'^{-1} U^T eta; dL/db = lambda and
// dL/dA_ij = -lambda_i x_j.  With the forward solve's W (backward_y_impl):
// Theorem 3.1's A^{-1} = A~^{-1} - W K^{-1} V^T A~^{-1} transposes to
// A^{-T} = A~^{-T} (I - V K^{-T} W^T), one system with A~^T per pass.
#include "sai_internal.hpp"

#include <map>
#include <mutex>

namespace sai {
namespace {

constexpr int NT = 256;
constexpr int NBR = 1024;

__global__ void k_smw_gather(int s, int kk, const int32_t* __restrict__ D, const double* __restrict__ Y,
                             double* __restrict__ K, double* __restrict__ rhs) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= s * s) return;
  const int d = t / s, e = t % s;
  K[t] = (d == e ? 1.0 : 0.0) + Y[(int64_t)D[d] * kk + 1 + e];
  if (e == 0) rhs[d] = Y[(int64_t)D[d] * kk];
}

// x_i = Y[i,0] - sum_e Y[i, 1+e] z_e
__global__ void k_smw_apply(int64_t n, int s, int kk, const double* __restrict__ Y,
                            const double* __restrict__ z, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    double acc = Y[i * kk];
    for (int e = 0; e < s; ++e) acc -= Y[i * kk + 1 + e] * z[e];
    x[i] = acc;
  }
}

// partial sums of ||b - A~ x - U x(j)||^2 and ||b||^2
__global__ void __launch_bounds__(NT) k_residual(int64_t n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci,
                                                 const double* __restrict__ v,
                                                 const int32_t* __restrict__ urp,
                                                 const int32_t* __restrict__ ucol,
                                                 const double* __restrict__ uval,
                                                 const int32_t* __restrict__ D,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[NT / WAVE];
  double a1 = 0.0, a2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    double y = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) y += v[e] * x[ci[e]];
    for (int32_t e = urp[i]; e < urp[i + 1]; ++e) y += uval[e] * x[D[ucol[e]]];
    const double r = b[i] - y;
    a1 += r * r;
    a2 += b[i] * b[i];
  }
  a1 = block_sum<NT>(a1, red);
  a2 = block_sum<NT>(a2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a1;
    part[NBR + blockIdx.x] = a2;
  }
}

__global__ void __launch_bounds__(NT) k_residual_final(int nb, const double* part, double* out) {
  __shared__ double red[NT / WAVE];
  double a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) {
    a1 += part[i];
    a2 += part[NBR + i];
  }
  a1 = block_sum<NT>(a1, red);
  a2 = block_sum<NT>(a2, red);
  if (threadIdx.x == 0) {
    out[0] = a1;
    out[1] = a2;
  }
}

// y = a x (y may alias x)
__global__ void k_scale_copy(int64_t n, double a, const double* x, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) y[i] = a * x[i];
}

// R = [b | U] (row-major n x (s+1))
__global__ void k_rhs_bu(int64_t n, int s, const double* __restrict__ b,
                         const int32_t* __restrict__ urp, const int32_t* __restrict__ ucol,
                         const double* __restrict__ uval, double* __restrict__ R) {
  const int kk = s + 1;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    R[i * kk] = b[i];
    for (int d = 0; d < s; ++d) R[i * kk + 1 + d] = 0.0;
    for (int32_t e = urp[i]; e < urp[i + 1]; ++e) R[i * kk + 1 + ucol[e]] = uval[e];
  }
}

// R = [g | V] with V = (e_{j_1}..e_{j_s})
__global__ void k_rhs_gv(int64_t n, int s, const double* __restrict__ g, double* __restrict__ R) {
  const int kk = s + 1;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    R[i * kk] = g[i];
    for (int d = 0; d < s; ++d) R[i * kk + 1 + d] = 0.0;
  }
}
__global__ void k_set_units(int s, const int32_t* D, double* R) {
  const int d = blockIdx.x * NT + threadIdx.x;
  if (d < s) R[(int64_t)D[d] * (s + 1) + 1 + d] = 1.0;
}

// correction solves: R = U - A~ W for the auxiliary columns (c-refinement).  One
// thread per (row i, column d), consecutive threads on consecutive columns of a
// row, so that the gathered rows of Y are read whole by neighbouring lanes.
__global__ void k_aux_residual(int64_t n, int s, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ ci, const double* __restrict__ v,
                               const int32_t* __restrict__ urp, const int32_t* __restrict__ ucol,
                               const double* __restrict__ uval, const double* __restrict__ Y,
                               double* __restrict__ R) {
  const int kk = s + 1;
  const int64_t ns = n * s;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < ns; t += (int64_t)gridDim.x * NT) {
    const int64_t i = t / s;
    const int d = (int)(t % s);
    double y = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) y += v[e] * Y[(int64_t)ci[e] * kk + 1 + d];
    double r = -y;
    for (int32_t e = urp[i]; e < urp[i + 1]; ++e)
      if (ucol[e] == d) r += uval[e];
    R[t] = r;
  }
}
// adjoint correction solves: R = V - A~^T Z for the auxiliary columns, with A~^T
// given as the CSC of A~ and V = (e_{j_1} .. e_{j_s}) (added by k_add_units);
// the thread map of k_aux_residual
__global__ void k_aux_residual_t(int64_t n, int s, const int32_t* __restrict__ cp,
                                 const int32_t* __restrict__ ri, const double* __restrict__ cv,
                                 const double* __restrict__ Y, double* __restrict__ R) {
  const int kk = s + 1;
  const int64_t ns = n * s;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < ns; t += (int64_t)gridDim.x * NT) {
    const int64_t i = t / s;
    const int d = (int)(t % s);
    double y = 0.0;
    for (int32_t e = cp[i]; e < cp[i + 1]; ++e) y += cv[e] * Y[(int64_t)ri[e] * kk + 1 + d];
    R[t] = -y;
  }
}
__global__ void k_add_units(int s, const int32_t* D, double* R) {
  const int d = blockIdx.x * NT + threadIdx.x;
  if (d < s) R[(int64_t)D[d] * s + d] += 1.0;
}

__global__ void k_aux_add(int64_t n, int s, const double* __restrict__ dW, double* __restrict__ Y) {
  const int kk = s + 1;
  const int64_t ns = n * s;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < ns; t += (int64_t)gridDim.x * NT)
    Y[(t / s) * kk + 1 + t % s] += dW[t];
}

// P = U^T Y (s x kk): block b accumulates the U entries of its row range in row
// order for the columns c0 .. c0+cw-1 of Y (s x cw doubles of LDS); lane e owns
// columns c0 + e, c0 + e + 64, ...  Then the partials are summed over blocks in
// order.  UTY_LDS bounds the LDS of one launch; wider blocks take several.
constexpr int UTY_ROWS = 4096;
constexpr int UTY_LDS = 6144;  // doubles (48 KB)
__global__ void __launch_bounds__(64) k_uty_partial(int64_t n, int s, int kk, int c0, int cw,
                                                    const int32_t* __restrict__ urp,
                                                    const int32_t* __restrict__ ucol,
                                                    const double* __restrict__ uval,
                                                    const double* __restrict__ Y,
                                                    double* __restrict__ part) {
  extern __shared__ double acc[];  // s * cw
  const int e = threadIdx.x;
  for (int t = e; t < s * cw; t += 64) acc[t] = 0.0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * UTY_ROWS;
  const int64_t i1 = std::min<int64_t>(n, i0 + UTY_ROWS);
  for (int64_t i = i0; i < i1; ++i) {
    for (int32_t q = urp[i]; q < urp[i + 1]; ++q) {
      const int d = ucol[q];
      const double u = uval[q];
      for (int c = e; c < cw; c += 64) acc[d * cw + c] += u * Y[i * kk + c0 + c];
    }
  }
  __syncthreads();
  for (int t = e; t < s * cw; t += 64)
    part[((int64_t)blockIdx.x * s + t / cw) * kk + c0 + t % cw] = acc[t];
}
__global__ void k_uty_final(int nb, int s, int kk, const double* __restrict__ part,
                            double* __restrict__ P) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= s * kk) return;
  double a = 0.0;
  for (int b = 0; b < nb; ++b) a += part[(int64_t)b * s * kk + t];
  P[t] = a;
}
// K' = I + P[:, 1:], rhs = P[:, 0]
__global__ void k_kprime(int s, int kk, const double* P, double* K, double* rhs) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= s * s) return;
  const int d = t / s, e = t % s;
  K[t] = (d == e ? 1.0 : 0.0) + P[d * kk + 1 + e];
  if (e == 0) rhs[d] = P[d * kk];
}

__global__ void k_grad_a(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const double* __restrict__ lam, const double* __restrict__ x,
                         double* __restrict__ ga) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double l = lam[i];
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) ga[e] = -l * x[ci[e]];
  }
}

// ---- the adjoint from the forward solve's W ----------------------------------------

// part[b][c0 + c] = sum over the rows of block b of W[i, c0 + c] v[i], W = Y[:, 1..s]
// (row stride s + 1): thread t takes column c0 + t % cw and the rows i0 + t / cw,
// i0 + t / cw + G, ... (G = NT / cw row groups, added in order afterwards)
constexpr int WTV_ROWS = 2048;
__global__ void __launch_bounds__(NT) k_wtv_partial(int64_t n, int s, int c0, int cw,
                                                    const double* __restrict__ Y,
                                                    const double* __restrict__ v,
                                                    double* __restrict__ part) {
  __shared__ double red[NT];
  const int G = NT / cw;
  const int t = threadIdx.x, c = t % cw, g = t / cw;
  const int kk = s + 1;
  const int64_t i0 = (int64_t)blockIdx.x * WTV_ROWS;
  const int64_t i1 = std::min<int64_t>(n, i0 + WTV_ROWS);
  double a = 0.0;
  if (g < G)
    for (int64_t i = i0 + g; i < i1; i += G) a += Y[i * kk + 1 + c0 + c] * v[i];
  red[t] = a;
  __syncthreads();
  if (t < cw) {
    double r = 0.0;
    for (int u = 0; u < G; ++u) r += red[u * cw + t];
    part[(int64_t)blockIdx.x * s + c0 + t] = r;
  }
}

// P[e] = sum over blocks b < nb of part[b s + e]: block e; thread t adds the blocks
// t, t + NT, ... in order, then a fixed-order block sum
__global__ void __launch_bounds__(NT) k_cols_final(int nb, int s, const double* __restrict__ part,
                                                   double* __restrict__ P) {
  __shared__ double red[NT / WAVE];
  const int e = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) a += part[(int64_t)b * s + e];
  a = block_sum<NT>(a, red);
  if (threadIdx.x == 0) P[e] = a;
}

// K^T (row-major s x s) with K = I + V^T W: K^T[e][d] = delta_de + W[j_d, e]
__global__ void k_kt(int s, int kk, const int32_t* __restrict__ D, const double* __restrict__ Y,
                     double* __restrict__ Kt) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= s * s) return;
  const int e = t / s, d = t % s;
  Kt[t] = (d == e ? 1.0 : 0.0) + Y[(int64_t)D[d] * kk + 1 + e];
}

// v(j_d) -= z_d, i.e. v -= V z (the j_d are distinct)
__global__ void k_sub_units(int s, const int32_t* __restrict__ D, const double* __restrict__ z,
                            double* __restrict__ v) {
  const int d = blockIdx.x * NT + threadIdx.x;
  if (d < s) v[D[d]] -= z[d];
}

// rho = g - A~^T lam, with A~^T given as the CSC of A~ (row j of A~^T = column j)
__global__ void k_resid_t(int64_t n, const int32_t* __restrict__ cp, const int32_t* __restrict__ ri,
                          const double* __restrict__ cv, const double* __restrict__ g,
                          const double* __restrict__ lam, double* __restrict__ rho) {
  for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < n; j += (int64_t)gridDim.x * NT) {
    double y = 0.0;
    for (int32_t e = cp[j]; e < cp[j + 1]; ++e) y += cv[e] * lam[ri[e]];
    rho[j] = g[j] - y;
  }
}

// out[0] = sum over d of (r(j_d) + q_d)^2 - r(j_d)^2, in order (||r + V q||^2 - ||r||^2)
__global__ void k_amp_terms(int s, const int32_t* __restrict__ D, const double* __restrict__ r,
                            const double* __restrict__ q, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0;
  for (int d = 0; d < s; ++d) {
    const double v = r[D[d]];
    a += (v + q[d]) * (v + q[d]) - v * v;
  }
  out[0] = a;
}

// y += d
__global__ void k_add_vec(int64_t n, const double* __restrict__ d, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) y[i] += d[i];
}

unsigned rows_grid(int64_t n) { return grid_for(n, NT, 8192); }

std::vector<double> thresholds(double bnorm, int s, double eps, double c) {
  std::vector<double> t(s + 1);
  t[0] = 0.5 * eps * bnorm;
  for (int d = 1; d <= s; ++d) t[d] = eps * bnorm / (2.0 * std::sqrt((double)s) * c);
  return t;
}

}  // namespace

void smw_recover(const sai_split_s* sp, const double* Y, double* x, double* c_host, hipStream_t st) {
  const Allocator al{sp->al.a, st};
  const int s = sp->s, kk = s + 1;
  const int64_t n = sp->n;
  SAI_PROF("smw_recover", st);
  if (s == 0) {
    hipLaunchKernelGGL(k_smw_apply, dim3(rows_grid(n)), dim3(NT), 0, st, n, 0, 1, Y,
                       (const double*)nullptr, x);
    LAUNCH_CHECK();
    if (c_host) *c_host = 0.0;
    HIPC(hipStreamSynchronize(st));
    return;
  }
  DBuf<double> K(&al, (size_t)s * s), z(&al, (size_t)s);
  hipLaunchKernelGGL(k_smw_gather, dim3(grid_for(s * s, NT)), dim3(NT), 0, st, s, kk,
                     sp->dense_cols.p, Y, K.p, z.p);
  LAUNCH_CHECK();
  if (!dense_lu_solve(K.p, z.p, s, 1, al, st))
    SAI_THROW(SAI_ESINGULAR, "I + V^T W is singular (zero pivot)");
  hipLaunchKernelGGL(k_smw_apply, dim3(rows_grid(n)), dim3(NT), 0, st, n, s, kk, Y,
                     (const double*)z.p, x);
  LAUNCH_CHECK();
  if (c_host) {
    std::vector<double> hz(s);
    HIPC(hipMemcpyAsync(hz.data(), z.p, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double a = 0.0;
    for (double v : hz) a += v * v;
    *c_host = std::sqrt(a);
  }
  HIPC(hipStreamSynchronize(st));
}

// ---- SMW recovery without allocation -------------------------------------------
// For callers that cannot allocate device memory: K (s x s), z (s) and the LU
// pivot flag live in this file-scope array (one copy per GPU, held until the
// process ends).  Every call on a GPU uses that GPU's copy, so calls that
// overlap on one GPU race; each call clears the flag it reads and overwrites
// K and z before reading them.
constexpr size_t SMW_SCR_K = (size_t)SMW_NOALLOC_SMAX * SMW_NOALLOC_SMAX;  // doubles
constexpr size_t SMW_SCR_Z = SMW_SCR_K;                                        // offset of z
constexpr size_t SMW_SCR_FLAG = SMW_SCR_K + SMW_NOALLOC_SMAX;                  // offset of the flag
constexpr size_t SMW_SCR_DOUBLES = SMW_SCR_FLAG + 32;                         // 33,536 bytes
static __device__ __align__(256) double scratch[SMW_SCR_DOUBLES];

namespace {
// device address of `scratch` per device, resolved once per device with that
// device current (the host-side name is not a device address)
std::mutex scr_mu;
std::map<int, double*> scr_ptr;

double* scratch_ptr() {
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(scr_mu);
  auto it = scr_ptr.find(dev);
  if (it != scr_ptr.end()) return it->second;
  double* p = nullptr;
  HIPC(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
  if (!p) SAI_THROW(SAI_EHIP, "no device address for the SMW scratch array");
  scr_ptr[dev] = p;
  return p;
}
}  // namespace

void smw_recover_noalloc(const sai_split_s* sp, const double* Y, double* x, double* c_host,
                         hipStream_t st) {
  const int s = sp->s, kk = s + 1;
  const int64_t n = sp->n;
  if (s > SMW_NOALLOC_SMAX)
    SAI_THROW(SAI_ETOOBIG, "s = %d exceeds %d, the limit of the allocation-free SMW recovery", s,
              SMW_NOALLOC_SMAX);
  if (s == 0) {
    hipLaunchKernelGGL(k_smw_apply, dim3(rows_grid(n)), dim3(NT), 0, st, n, 0, 1, Y,
                       (const double*)nullptr, x);
    LAUNCH_CHECK();
    if (c_host) *c_host = 0.0;
    HIPC(hipStreamSynchronize(st));
    return;
  }
  double* base = scratch_ptr();
  double* K = base;
  double* z = base + SMW_SCR_Z;
  int* fail = reinterpret_cast<int*>(base + SMW_SCR_FLAG);
  fill_i32(fail, 0, 1, st);  // a kernel, not a memset node
  hipLaunchKernelGGL(k_smw_gather, dim3(grid_for(s * s, NT)), dim3(NT), 0, st, s, kk, sp->dense_cols.p, Y,
                     K, z);
  LAUNCH_CHECK();
  launch_dense_lu(K, z, s, 1, fail, st);
  int hfail = 0;
  HIPC(hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (hfail) SAI_THROW(SAI_ESINGULAR, "I + V^T W is singular (zero pivot)");
  hipLaunchKernelGGL(k_smw_apply, dim3(rows_grid(n)), dim3(NT), 0, st, n, s, kk, Y, (const double*)z, x);
  LAUNCH_CHECK();
  if (c_host) {
    double hz[SMW_NOALLOC_SMAX];
    HIPC(hipMemcpyAsync(hz, z, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double a = 0.0;
    for (int d = 0; d < s; ++d) a += hz[d] * hz[d];
    *c_host = std::sqrt(a);
  }
  HIPC(hipStreamSynchronize(st));
}

double residual_impl(const sai_split_s* sp, const double* b, const double* x, hipStream_t st) {
  const Allocator al{sp->al.a, st};
  const int64_t n = sp->n;
  DBuf<double> part(&al, 2 * NBR + 2);
  const unsigned nb = grid_for(n, NT, NBR);
  SAI_PROF("residual_check", st);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(NT), 0, st, n, sp->t_row_ptr.p, sp->t_col_idx.p,
                     sp->t_val.p, sp->u_row_ptr.p, sp->u_col.p, sp->u_val.p, sp->dense_cols.p, b, x,
                     part.p);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(NT), 0, st, (int)nb, part.p, part.p + 2 * NBR);
  LAUNCH_CHECK();
  double h[2];
  HIPC(hipMemcpyAsync(h, part.p + 2 * NBR, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
}

void solve_impl(const sai_split_s* sp, const sai_precond_s* pc, const double* b, double* x,
                const sai_solve_opts& o, hipStream_t st, sai_solve_stats* stats, double* y_out) {
  const Allocator al{sp->al.a, st};
  const int s = sp->s, kk = s + 1;
  const int64_t n = sp->n;
  EventTimer t_solve, t_smw, t_chk;
  // the Krylov solutions [y, W] go to the caller's y_out when given
  DBuf<double> R(&al, (size_t)n * kk), Ybuf;
  if (!y_out) Ybuf.alloc(&al, (size_t)n * kk);
  double* const Y = y_out ? y_out : Ybuf.p;
  // Section 4's scaling (equilibrate): solve with alpha b, alpha = rho / ||b||,
  // rho = ||A||_F / sqrt(n) (||A||_F^2 = ||A~||_F^2 + ||U||_F^2), x scaled back
  double alpha = 1.0;
  DBuf<double> bs;
  if (o.equilibrate) {
    const double fa = dev_norm2(sp->t_val.p, sp->nnz_t, 1, al, st);
    const double fu = sp->nnz_u > 0 ? dev_norm2(sp->u_val.p, sp->nnz_u, 1, al, st) : 0.0;
    const double rho = std::sqrt((fa * fa + fu * fu) / (double)n);
    const double b0 = dev_norm2(b, n, 1, al, st);
    if (b0 > 0.0 && rho > 0.0) {
      alpha = rho / b0;
      bs.alloc(&al, (size_t)n);
      hipLaunchKernelGGL(k_scale_copy, dim3(rows_grid(n)), dim3(NT), 0, st, n, alpha, b, bs.p);
      LAUNCH_CHECK();
      b = bs.p;
    }
  }
  hipLaunchKernelGGL(k_rhs_bu, dim3(rows_grid(n)), dim3(NT), 0, st, n, s, b, sp->u_row_ptr.p,
                     sp->u_col.p, sp->u_val.p, R.p);
  LAUNCH_CHECK();
  const double bnorm = dev_norm2(b, n, 1, al, st);
  std::vector<double> thr = thresholds(bnorm, s, o.eps, 1.0);
  std::vector<int32_t> its(kk, 0), sts(kk, 0);
  t_solve.start(st);
  int code = krylov_impl(sp, pc, 0, kk, R.p, Y, thr.data(), o, st, its.data(), sts.data());
  t_solve.stop(st);
  double c = 0.0;
  t_smw.start(st);
  smw_recover(sp, Y, x, &c, st);
  t_smw.stop(st);
  t_chk.start(st);
  double rr = residual_impl(sp, b, x, st);
  t_chk.stop(st);
  float extra_ms = 0.0f;
  if (o.c_mode == SAI_C_ONE_THEN_REFINE && rr >= o.eps && c > 1.0 && s > 0 && code == SAI_OK) {
    // continue the auxiliary solves to the thresholds with the computed c
    EventTimer t_ref;
    t_ref.start(st);
    std::vector<double> thr2 = thresholds(bnorm, s, o.eps, c);
    DBuf<double> Raux(&al, (size_t)n * s), dW(&al, (size_t)n * s);
    hipLaunchKernelGGL(k_aux_residual, dim3(grid_for(n * s, NT, 8192)), dim3(NT), 0, st, n, s, sp->t_row_ptr.p,
                       sp->t_col_idx.p, sp->t_val.p, sp->u_row_ptr.p, sp->u_col.p, sp->u_val.p,
                       Y, Raux.p);
    LAUNCH_CHECK();
    std::vector<int32_t> its2(s, 0), sts2(s, 0);
    code = krylov_impl(sp, pc, 0, s, Raux.p, dW.p, thr2.data() + 1, o, st, its2.data(), sts2.data());
    hipLaunchKernelGGL(k_aux_add, dim3(grid_for(n * s, NT, 8192)), dim3(NT), 0, st, n, s, dW.p, Y);
    LAUNCH_CHECK();
    for (int d = 0; d < s; ++d) its[d + 1] += its2[d];
    smw_recover(sp, Y, x, &c, st);
    rr = residual_impl(sp, b, x, st);
    t_ref.stop(st);
    extra_ms = t_ref.ms();
  }
  if (alpha != 1.0) {
    hipLaunchKernelGGL(k_scale_copy, dim3(rows_grid(n)), dim3(NT), 0, st, n, 1.0 / alpha, (const double*)x, x);
    LAUNCH_CHECK();
    HIPC(hipStreamSynchronize(st));
  }
  if (stats) {
    stats->s = s;
    stats->status = code;
    int mx = 0;
    for (int q = 0; q < kk; ++q) mx = std::max(mx, its[q]);
    stats->iters_max = mx;
    if (stats->iters)
      for (int q = 0; q < kk; ++q) stats->iters[q] = its[q];
    stats->rr = rr;
    stats->a = rr / o.eps;
    stats->c = c;
    stats->t_solve_ms = t_solve.ms() + extra_ms;
    stats->t_smw_ms = t_smw.ms();
    stats->t_check_ms = t_chk.ms();
  }
  if (code != SAI_OK) throw Error{code, "Krylov solve did not converge on every column"};
}

void backward_impl(const sai_split_s* sp, const sai_precond_s* pc, const double* x, const double* gx,
                   double* gb, double* ga, const sai_solve_opts& o, hipStream_t st,
                   sai_solve_stats* stats) {
  const Allocator al{sp->al.a, st};
  const int s = sp->s, kk = s + 1;
  const int64_t n = sp->n;
  EventTimer t_solve, t_smw;
  DBuf<double> R(&al, (size_t)n * kk), Y(&al, (size_t)n * kk), lam(&al, (size_t)n);
  hipLaunchKernelGGL(k_rhs_gv, dim3(rows_grid(n)), dim3(NT), 0, st, n, s, gx, R.p);
  LAUNCH_CHECK();
  if (s > 0) {
    hipLaunchKernelGGL(k_set_units, dim3(grid_for(s, NT)), dim3(NT), 0, st, s, sp->dense_cols.p, R.p);
    LAUNCH_CHECK();
  }
  const double gnorm = dev_norm2(gx, n, 1, al, st);
  std::vector<double> thr = thresholds(gnorm, s, o.eps, 1.0);
  std::vector<int32_t> its(kk, 0), sts(kk, 0);
  t_solve.start(st);
  int code = krylov_impl(sp, pc, 1, kk, R.p, Y.p, thr.data(), o, st, its.data(), sts.data());
  t_solve.stop(st);
  t_smw.start(st);
  // lambda = eta - Z (I + U^T Z)^{-1} U^T eta; returns c' = ||(I + U^T Z)^{-1} U^T eta||
  auto recover = [&]() -> double {
    if (s == 0) {
      hipLaunchKernelGGL(k_smw_apply, dim3(rows_grid(n)), dim3(NT), 0, st, n, 0, 1, Y.p,
                         (const double*)nullptr, lam.p);
      LAUNCH_CHECK();
      return 0.0;
    }
    const int64_t nb = (n + UTY_ROWS - 1) / UTY_ROWS;
    DBuf<double> part(&al, (size_t)nb * s * kk), P(&al, (size_t)s * kk), K(&al, (size_t)s * s),
        w(&al, (size_t)s);
    const int cw = std::max(1, std::min(kk, UTY_LDS / s));
    for (int c0 = 0; c0 < kk; c0 += cw) {
      const int w = std::min(cw, kk - c0);
      hipLaunchKernelGGL(k_uty_partial, dim3((unsigned)nb), dim3(64), sizeof(double) * s * w, st, n, s,
                         kk, c0, w, sp->u_row_ptr.p, sp->u_col.p, sp->u_val.p, Y.p, part.p);
      LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_uty_final, dim3(grid_for(s * kk, NT)), dim3(NT), 0, st, (int)nb, s, kk, part.p,
                       P.p);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_kprime, dim3(grid_for(s * s, NT)), dim3(NT), 0, st, s, kk, P.p, K.p, w.p);
    LAUNCH_CHECK();
    if (!dense_lu_solve(K.p, w.p, s, 1, al, st))
      SAI_THROW(SAI_ESINGULAR, "I + U^T Z is singular (zero pivot)");
    hipLaunchKernelGGL(k_smw_apply, dim3(rows_grid(n)), dim3(NT), 0, st, n, s, kk, Y.p,
                       (const double*)w.p, lam.p);
    LAUNCH_CHECK();
    std::vector<double> hw(s);
    HIPC(hipMemcpyAsync(hw.data(), w.p, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double a = 0.0;
    for (double v : hw) a += v * v;
    return std::sqrt(a);
  };
  double cprime = recover();
  if (o.c_mode == SAI_C_ONE_THEN_REFINE && cprime > 1.0 && s > 0 && code == SAI_OK) {
    // the theorem's condition with the computed c': continue the s auxiliary
    // solves (correction solves on V - A~^T Z) to eps ||g|| / (2 sqrt(s) c')
    std::vector<double> thr2 = thresholds(gnorm, s, o.eps, cprime);
    DBuf<double> Raux(&al, (size_t)n * s), dZ(&al, (size_t)n * s);
    hipLaunchKernelGGL(k_aux_residual_t, dim3(grid_for(n * s, NT, 8192)), dim3(NT), 0, st, n, s, sp->t_col_ptr.p,
                       sp->t_row_idx.p, sp->t_cval.p, Y.p, Raux.p);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_add_units, dim3(grid_for(s, NT)), dim3(NT), 0, st, s, sp->dense_cols.p,
                       Raux.p);
    LAUNCH_CHECK();
    std::vector<int32_t> its2(s, 0), sts2(s, 0);
    code = krylov_impl(sp, pc, 1, s, Raux.p, dZ.p, thr2.data() + 1, o, st, its2.data(), sts2.data());
    hipLaunchKernelGGL(k_aux_add, dim3(grid_for(n * s, NT, 8192)), dim3(NT), 0, st, n, s, dZ.p, Y.p);
    LAUNCH_CHECK();
    for (int d = 0; d < s; ++d) its[d + 1] += its2[d];
    cprime = recover();
  }
  if (gb) HIPC(hipMemcpyAsync(gb, lam.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  if (ga) {
    hipLaunchKernelGGL(k_grad_a, dim3(rows_grid(n)), dim3(NT), 0, st, n, sp->a_row_ptr.p,
                       sp->a_col_idx.p, (const double*)lam.p, x, ga);
    LAUNCH_CHECK();
  }
  t_smw.stop(st);
  HIPC(hipStreamSynchronize(st));
  if (stats) {
    stats->s = s;
    stats->status = code;
    int mx = 0;
    for (int q = 0; q < kk; ++q) mx = std::max(mx, its[q]);
    stats->iters_max = mx;
    if (stats->iters)
      for (int q = 0; q < kk; ++q) stats->iters[q] = its[q];
    stats->rr = 0.0;
    stats->a = 0.0;
    stats->c = cprime;
    stats->t_solve_ms = t_solve.ms();
    stats->t_smw_ms = t_smw.ms();
    stats->t_check_ms = 0.0f;
  }
  if (code != SAI_OK) throw Error{code, "adjoint Krylov solve did not converge on every column"};
}

}  // namespace sai

namespace sai {

// Adjoint from the forward solve's W = Y[:, 1..s] (approximately A~^{-1} U).
// A^{-T} = A~^{-T} (I - V K^{-T} W^T), K = I + V^T W, so each pass solves one
// system A~^T d = r - V K^{-T} W^T r (M^T as right preconditioner) and adds d
// to lambda; r is grad_x, then the true residual grad_x - A~^T lambda -
// V (U^T lambda).  After a pass the true residual is (I + V W^T) r_s - V R^T d
// (r_s the solve's residual, R = U - A~ W the forward's auxiliary residuals:
// W's own error, which usually keeps the first pass above eps and which the
// next pass removes).  The first solve stops at (eps/2)||g||, each later one
// at (eps/2)||g|| / a with a = max(1, ||(I + V W^T) r_s|| / ||r_s||) of the
// pass before; passes stop once the true residual is below eps ||g||.
void backward_y_impl(const sai_split_s* sp, const sai_precond_s* pc, const double* x, const double* Y,
                     const double* gx, double* gb, double* ga, const sai_solve_opts& o, hipStream_t st,
                     sai_solve_stats* stats) {
  constexpr int PASSES = 4;
  const Allocator al{sp->al.a, st};
  const int s = sp->s, kk = s + 1;
  const int64_t n = sp->n;
  if (s > 0 && !Y) SAI_THROW(SAI_EINVAL, "Y (the forward solutions [y, W]) is required when s > 0");
  EventTimer t_all, t_solve, t_chk;
  float solve_ms = 0.0f, chk_ms = 0.0f;
  t_all.start(st);
  DBuf<double> lam(&al, (size_t)n), res(&al, (size_t)n), rhs(&al, (size_t)n), del(&al, (size_t)n),
      rs(&al, (size_t)n);
  const int64_t nbw = (n + WTV_ROWS - 1) / WTV_ROWS, nbu = (n + UTY_ROWS - 1) / UTY_ROWS;
  const int sm = std::max(s, 1);
  DBuf<double> part(&al, (size_t)std::max(nbw, nbu) * sm), P(&al, (size_t)sm), Kt(&al, (size_t)sm * sm);
  const double gnorm = dev_norm2(gx, n, 1, al, st);
  if (!std::isfinite(gnorm)) SAI_THROW(SAI_EINVAL, "grad_x has a non-finite entry");
  // out = v - V K^{-T} W^T v; returns ||K^{-T} W^T v|| when `norm`
  auto correct = [&](const double* v, double* out, bool norm) -> double {
    SAI_PROF("adjoint_correction", st);
    hipLaunchKernelGGL(k_scale_copy, dim3(rows_grid(n)), dim3(NT), 0, st, n, 1.0, v, out);
    LAUNCH_CHECK();
    if (s == 0) return 0.0;
    for (int c0 = 0; c0 < s; c0 += NT) {
      const int cw = std::min(NT, s - c0);
      hipLaunchKernelGGL(k_wtv_partial, dim3((unsigned)nbw), dim3(NT), 0, st, n, s, c0, cw, Y, v, part.p);
      LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_cols_final, dim3(s), dim3(NT), 0, st, (int)nbw, s, (const double*)part.p, P.p);
    hipLaunchKernelGGL(k_kt, dim3(grid_for(s * s, NT)), dim3(NT), 0, st, s, kk, sp->dense_cols.p, Y, Kt.p);
    LAUNCH_CHECK();
    if (!dense_lu_solve(Kt.p, P.p, s, 1, al, st))
      SAI_THROW(SAI_ESINGULAR, "I + V^T W is singular (zero pivot)");
    hipLaunchKernelGGL(k_sub_units, dim3(grid_for(s, NT)), dim3(NT), 0, st, s, sp->dense_cols.p,
                       (const double*)P.p, out);
    LAUNCH_CHECK();
    if (!norm) return 0.0;
    std::vector<double> hz(s);
    HIPC(hipMemcpyAsync(hz.data(), P.p, sizeof(double) * s, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double a = 0.0;
    for (double v : hz) a += v * v;
    return std::sqrt(a);
  };
  // res = g - A~^T lam - V (U^T lam); returns ||res||
  auto true_residual = [&]() -> double {
    SAI_PROF("adjoint_residual", st);
    hipLaunchKernelGGL(k_resid_t, dim3(rows_grid(n)), dim3(NT), 0, st, n, sp->t_col_ptr.p, sp->t_row_idx.p,
                       sp->t_cval.p, gx, (const double*)lam.p, res.p);
    LAUNCH_CHECK();
    if (s > 0) {
      hipLaunchKernelGGL(k_uty_partial, dim3((unsigned)nbu), dim3(64), sizeof(double) * s, st, n, s, 1, 0, 1,
                         sp->u_row_ptr.p, sp->u_col.p, sp->u_val.p, (const double*)lam.p, part.p);
      LAUNCH_CHECK();
      hipLaunchKernelGGL(k_cols_final, dim3(s), dim3(NT), 0, st, (int)nbu, s, (const double*)part.p, P.p);
      hipLaunchKernelGGL(k_sub_units, dim3(grid_for(s, NT)), dim3(NT), 0, st, s, sp->dense_cols.p,
                         (const double*)P.p, res.p);
      LAUNCH_CHECK();
    }
    return dev_norm2(res.p, n, 1, al, st);
  };
  // a = max(1, ||(I + V W^T) r_s|| / ||r_s||) for the last solve, r_s = rhs - A~^T del
  auto solve_amplification = [&]() -> double {
    SAI_PROF("adjoint_correction", st);
    hipLaunchKernelGGL(k_resid_t, dim3(rows_grid(n)), dim3(NT), 0, st, n, sp->t_col_ptr.p, sp->t_row_idx.p,
                       sp->t_cval.p, (const double*)rhs.p, (const double*)del.p, rs.p);
    LAUNCH_CHECK();
    const double nrs = dev_norm2(rs.p, n, 1, al, st);
    if (s == 0 || !(nrs > 0.0)) return 1.0;
    for (int c0 = 0; c0 < s; c0 += NT) {
      const int cw = std::min(NT, s - c0);
      hipLaunchKernelGGL(k_wtv_partial, dim3((unsigned)nbw), dim3(NT), 0, st, n, s, c0, cw, Y,
                         (const double*)rs.p, part.p);
      LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_cols_final, dim3(s), dim3(NT), 0, st, (int)nbw, s, (const double*)part.p, P.p);
    hipLaunchKernelGGL(k_amp_terms, dim3(1), dim3(64), 0, st, s, sp->dense_cols.p, (const double*)rs.p,
                       (const double*)P.p, Kt.p);
    LAUNCH_CHECK();
    double extra = 0.0;
    HIPC(hipMemcpyAsync(&extra, Kt.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    return std::max(1.0, std::sqrt(std::max(0.0, nrs * nrs + extra)) / nrs);
  };
  HIPC(hipMemsetAsync(lam.p, 0, sizeof(double) * n, st));
  int code = SAI_OK, its = 0;
  double rr = 0.0, c = 0.0;
  if (gnorm > 0.0) {
    double thr = 0.5 * o.eps * gnorm;
    const double* src = gx;
    for (int pass = 1; pass <= PASSES; ++pass) {
      const double zn = correct(src, rhs.p, pass == 1);
      if (pass == 1) c = zn;
      int32_t it = 0, stc = 0;
      t_solve.start(st);
      const int kc = krylov_impl(sp, pc, 1, 1, rhs.p, del.p, &thr, o, st, &it, &stc);
      t_solve.stop(st);
      solve_ms += t_solve.ms();
      its += it;
      hipLaunchKernelGGL(k_add_vec, dim3(rows_grid(n)), dim3(NT), 0, st, n, (const double*)del.p, lam.p);
      LAUNCH_CHECK();
      t_chk.start(st);
      const double rn = true_residual();
      t_chk.stop(st);
      chk_ms += t_chk.ms();
      rr = rn / gnorm;
      if (rr < o.eps) {
        code = SAI_OK;
        break;
      }
      code = kc == SAI_EBREAKDOWN ? SAI_EBREAKDOWN : SAI_ENOCONV;
      if (kc == SAI_EBREAKDOWN || pass == PASSES) break;
      thr = 0.5 * o.eps * gnorm / solve_amplification();
      src = res.p;
    }
  }
  if (gb) HIPC(hipMemcpyAsync(gb, lam.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  if (ga) {
    hipLaunchKernelGGL(k_grad_a, dim3(rows_grid(n)), dim3(NT), 0, st, n, sp->a_row_ptr.p, sp->a_col_idx.p,
                       (const double*)lam.p, x, ga);
    LAUNCH_CHECK();
  }
  t_all.stop(st);
  HIPC(hipStreamSynchronize(st));
  if (stats) {
    stats->s = s;
    stats->status = code;
    stats->iters_max = its;
    if (stats->iters)
      for (int q = 0; q < kk; ++q) stats->iters[q] = q == 0 ? its : 0;
    stats->rr = rr;
    stats->a = rr / o.eps;
    stats->c = c;
    stats->t_solve_ms = solve_ms;
    stats->t_smw_ms = std::max(0.0f, t_all.ms() - solve_ms - chk_ms);
    stats->t_check_ms = chk_ms;
  }
  if (code != SAI_OK) throw Error{code, "adjoint residual not below eps after the correction passes"};
}

}  // namespace sai
