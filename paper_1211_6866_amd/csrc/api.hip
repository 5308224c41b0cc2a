// C ABI of libsai: argument checks, error translation and handle lifetime.
#include "sai_internal.hpp"

namespace sai {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }

}  // namespace sai

using sai::Allocator;
using sai::Error;

namespace {

template <class F>
int guarded(F&& f) {
  try {
    f();
    sai::set_last_error("");
    return SAI_OK;
  } catch (const Error& e) {
    sai::set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    sai::set_last_error("host allocation failed");
    return SAI_ENOMEM;
  } catch (...) {
    sai::set_last_error("unexpected exception");
    return SAI_EHIP;
  }
}

}  // namespace

extern "C" {

int sai_split(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx, const double* val,
              const sai_split_opts* opts, const sai_allocator* alloc, void* stream, sai_split_t** out) {
  if (!out) return SAI_EINVAL;
  *out = nullptr;
  sai_split_s* h = nullptr;
  int rc = guarded([&] {
    sai_split_opts o{10.0, 0, SAI_KEEP_NEAREST, nullptr, 0};
    if (opts) o = *opts;
    Allocator al;
    if (alloc) al.a = *alloc;
    al.stream = (hipStream_t)stream;
    h = new sai_split_s();
    sai::split_impl(n, nnz, row_ptr, col_idx, val, o, al, h);
  });
  if (rc == SAI_OK) *out = h;
  else delete h;
  return rc;
}

int sai_split_get_info(const sai_split_t* h, sai_split_info* info) {
  if (!h || !info) return SAI_EINVAL;
  info->n = h->n;
  info->s = h->s;
  info->p = h->p;
  info->keep = h->keep;
  info->nnz_a = h->nnz_a;
  info->nnz_t = h->nnz_t;
  info->nnz_u = h->nnz_u;
  info->t_row_ptr = h->t_row_ptr.p;
  info->t_col_idx = h->t_col_idx.p;
  info->t_val = h->t_val.p;
  info->t_col_ptr = h->t_col_ptr.p;
  info->t_row_idx = h->t_row_idx.p;
  info->t_cval = h->t_cval.p;
  info->dense_cols = h->dense_cols.p;
  info->u_row_ptr = h->u_row_ptr.p;
  info->u_col = h->u_col.p;
  info->u_val = h->u_val.p;
  return SAI_OK;
}

void sai_split_destroy(sai_split_t* h) { delete h; }

int sai_build(const sai_split_t* sp, const sai_build_opts* opts, void* stream, sai_precond_t** out,
              sai_build_stats* stats) {
  if (!sp || !opts || !out) return SAI_EINVAL;
  *out = nullptr;
  sai_precond_s* pc = nullptr;
  int rc = guarded([&] {
    pc = new sai_precond_s();
    sai::build_impl(sp, *opts, (hipStream_t)stream, pc, stats);
  });
  if (rc == SAI_OK) *out = pc;
  else delete pc;
  return rc;
}

int sai_precond_get_info(const sai_precond_t* h, sai_precond_info* info) {
  if (!h || !info) return SAI_EINVAL;
  info->n = h->n;
  info->precision = h->precision;
  info->nnz = h->nnz;
  info->col_ptr = h->col_ptr.p;
  info->row_idx = h->row_idx.p;
  info->cval = h->cval.p;
  info->row_ptr = h->row_ptr.p;
  info->col_idx = h->col_idx.p;
  info->val = h->val.p;
  info->j_ptr = h->j_ptr.p;
  info->j_idx = h->j_idx.p;
  info->i_ptr = h->i_ptr.p;
  info->i_idx = h->i_idx.p;
  info->m_full = h->m_full.p;
  info->res = h->res.p;
  return SAI_OK;
}

void sai_precond_destroy(sai_precond_t* h) { delete h; }

int sai_krylov(const sai_split_t* sp, const sai_precond_t* pc, int32_t transpose, int32_t k,
               const double* R, double* X, const double* thr, const sai_solve_opts* opts, void* stream,
               int32_t* iters, int32_t* status) {
  if (!sp || !pc || !R || !X || !thr || !opts) return SAI_EINVAL;
  int code = SAI_OK;
  int rc = guarded([&] {
    code = sai::krylov_impl(sp, pc, transpose, k, R, X, thr, *opts, (hipStream_t)stream, iters, status);
  });
  return rc != SAI_OK ? rc : code;
}

int sai_smw(const sai_split_t* sp, const double* Y, double* x, double* c, void* stream) {
  if (!sp || !Y || !x) return SAI_EINVAL;
  return guarded([&] { sai::smw_recover(sp, Y, x, c, (hipStream_t)stream); });
}

int sai_gather_offsets(const sai_precond_t* pc, int64_t* blk_off, int64_t* total, void* stream) {
  if (!pc || !blk_off) return SAI_EINVAL;
  return guarded([&] { sai::gather_offsets(pc, blk_off, total, (hipStream_t)stream); });
}

int sai_gather(const sai_split_t* sp, const sai_precond_t* pc, int32_t precision, const int64_t* blk_off,
               void* blocks, void* stream) {
  if (!sp || !pc || !blk_off || !blocks) return SAI_EINVAL;
  return guarded([&] { sai::gather_blocks(sp, pc, precision, blk_off, blocks, (hipStream_t)stream); });
}

int sai_smw_noalloc(const sai_split_t* sp, const double* Y, double* x, double* c, void* stream) {
  if (!sp || !Y || !x) return SAI_EINVAL;
  return guarded([&] { sai::smw_recover_noalloc(sp, Y, x, c, (hipStream_t)stream); });
}

int sai_residual(const sai_split_t* sp, const double* b, const double* x, double* rr, void* stream) {
  if (!sp || !b || !x || !rr) return SAI_EINVAL;
  return guarded([&] { *rr = sai::residual_impl(sp, b, x, (hipStream_t)stream); });
}

int sai_solve(const sai_split_t* sp, const sai_precond_t* pc, const double* b, double* x,
              const sai_solve_opts* opts, void* stream, sai_solve_stats* stats) {
  if (!sp || !pc || !b || !x || !opts) return SAI_EINVAL;
  return guarded([&] { sai::solve_impl(sp, pc, b, x, *opts, (hipStream_t)stream, stats); });
}

int sai_solve_y(const sai_split_t* sp, const sai_precond_t* pc, const double* b, double* x, double* Y,
                const sai_solve_opts* opts, void* stream, sai_solve_stats* stats) {
  if (!sp || !pc || !b || !x || !Y || !opts) return SAI_EINVAL;
  return guarded([&] { sai::solve_impl(sp, pc, b, x, *opts, (hipStream_t)stream, stats, Y); });
}

int sai_backward_y(const sai_split_t* sp, const sai_precond_t* pc, const double* x, const double* Y,
                   const double* grad_x, double* grad_b, double* grad_a_val, const sai_solve_opts* opts,
                   void* stream, sai_solve_stats* stats) {
  if (!sp || !pc || !x || !grad_x || !opts) return SAI_EINVAL;
  return guarded([&] {
    sai::backward_y_impl(sp, pc, x, Y, grad_x, grad_b, grad_a_val, *opts, (hipStream_t)stream, stats);
  });
}

int sai_backward(const sai_split_t* sp, const sai_precond_t* pc, const double* x, const double* grad_x,
                 double* grad_b, double* grad_a_val, const sai_solve_opts* opts, void* stream,
                 sai_solve_stats* stats) {
  if (!sp || !pc || !x || !grad_x || !opts) return SAI_EINVAL;
  return guarded([&] {
    sai::backward_impl(sp, pc, x, grad_x, grad_b, grad_a_val, *opts, (hipStream_t)stream, stats);
  });
}

const char* sai_strerror(int code) {
  switch (code) {
    case SAI_OK: return "ok";
    case SAI_EINVAL: return "invalid argument";
    case SAI_EZERODIAG: return "irregular column without a diagonal entry";
    case SAI_ESINGULAR: return "singular matrix";
    case SAI_ENOCONV: return "iteration limit reached";
    case SAI_EBREAKDOWN: return "BiCGStab breakdown";
    case SAI_ENOMEM: return "out of memory";
    case SAI_EHIP: return "HIP runtime error";
    case SAI_ETOOBIG: return "size exceeds a kernel limit";
    default: return "unknown error";
  }
}

const char* sai_last_error(void) { return sai::g_last_error.c_str(); }

// [A-Z0-9_]{1,63}
static bool tune_name_ok(const char* name) {
  if (!name || !*name) return false;
  size_t len = 0;
  for (const char* c = name; *c && len < 64; ++c, ++len)
    if (!((*c >= 'A' && *c <= 'Z') || (*c >= '0' && *c <= '9') || *c == '_')) return false;
  return len < 64;
}

int sai_tune_set(const char* name, int32_t value) {
  if (!tune_name_ok(name)) return SAI_EINVAL;
  sai::tune_set(name, value);
  return SAI_OK;
}

int sai_tune_get(const char* name, int32_t dflt, int32_t* value) {
  if (!tune_name_ok(name) || !value) return SAI_EINVAL;
  *value = sai::tune_get(name, dflt);
  return SAI_OK;
}

int sai_tune_clear(void) {
  sai::tune_clear();
  return SAI_OK;
}

int sai_memcpy_d2d(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return SAI_OK;
  if (!dst || !src) return SAI_EINVAL;
  return guarded([&] {
    HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    HIPC(hipStreamSynchronize((hipStream_t)stream));
  });
}

}  // extern "C"
