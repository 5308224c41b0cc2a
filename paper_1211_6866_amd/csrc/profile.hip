// Per-kernel event timing registry (enabled on request, for benchmarking).
#include <map>
#include <mutex>

#include "sai_internal.hpp"

namespace sai {
namespace {

struct Pending {
  std::string name;
  hipEvent_t a, b;
};

struct Registry {
  std::mutex mu;
  bool on = false;
  int mode = 0;
  std::string only;  // mode 3: record only the names that start with this
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<int64_t, double>> totals;

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    HIPC(hipEventCreate(&e));
    return e;
  }
  void resolve() {
    for (auto& p : pending) {
      HIPC(hipEventSynchronize(p.b));
      float ms = 0.0f;
      HIPC(hipEventElapsedTime(&ms, p.a, p.b));
      auto& t = totals[p.name];
      t.first += 1;
      t.second += ms;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};

Registry& reg() {
  static Registry r;
  return r;
}

}  // namespace

// Mode 2 records only the kernels that can dominate a step (the sparse products,
// the column solvers, the SPAI search and GMRES), to keep the event overhead low.
static bool hot_name(const char* n) {
  static const char* pre[] = {"bicg_spmm", "ls_qr", "spai", "gmres"};
  for (const char* p : pre)
    if (strncmp(n, p, strlen(p)) == 0) return true;
  return false;
}

ProfScope::ProfScope(const char* name, hipStream_t s) : st(s) {
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  if (!r.on) return;
  if (r.mode == 2 && !hot_name(name)) return;
  if (r.mode == 3 && strncmp(name, r.only.c_str(), r.only.size()) != 0) return;
  Pending p{name, r.get_event(), r.get_event()};
  HIPC(hipEventRecord(p.a, s));
  r.pending.push_back(p);
  slot = (int)r.pending.size() - 1;
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  if (slot < (int)r.pending.size()) (void)hipEventRecord(r.pending[slot].b, st);
}

}  // namespace sai

extern "C" {

int sai_profile_enable(int32_t on) {
  auto& r = sai::reg();
  std::lock_guard<std::mutex> g(r.mu);
  try {
    r.resolve();
  } catch (...) {
    return SAI_EHIP;
  }
  r.totals.clear();
  r.on = on != 0;
  r.mode = on;
  return SAI_OK;
}

int sai_profile_only(const char* prefix) {
  auto& r = sai::reg();
  std::lock_guard<std::mutex> g(r.mu);
  r.only = prefix ? prefix : "";
  return SAI_OK;
}

int sai_profile_count(void) {
  auto& r = sai::reg();
  std::lock_guard<std::mutex> g(r.mu);
  try {
    r.resolve();
  } catch (...) {
    return -1;
  }
  return (int)r.totals.size();
}

int sai_profile_get(int32_t i, char* name, int32_t name_cap, int64_t* launches, double* total_ms) {
  auto& r = sai::reg();
  std::lock_guard<std::mutex> g(r.mu);
  try {
    r.resolve();
  } catch (...) {
    return SAI_EHIP;
  }
  if (i < 0 || i >= (int)r.totals.size()) return SAI_EINVAL;
  auto it = r.totals.begin();
  std::advance(it, i);
  if (name && name_cap > 0) {
    strncpy(name, it->first.c_str(), (size_t)name_cap - 1);
    name[name_cap - 1] = 0;
  }
  if (launches) *launches = it->second.first;
  if (total_ms) *total_ms = it->second.second;
  return SAI_OK;
}

}  // extern "C"
