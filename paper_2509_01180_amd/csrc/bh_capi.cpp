// C ABI entry points (include/bh.h): argument checking, plan lifetime,
// device selection and dispatch to the kernel launchers.
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>

#include "bh_internal.h"

#include <algorithm>

namespace bh {

namespace {
thread_local std::string g_err;

// Make the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_error(BH_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(BH_EINVAL, e.what());
  } catch (...) {
    return set_error(BH_EINVAL, "unknown error");
  }
}

void free_band(DevBand& b) {
  for (void* q : {(void*)b.rec, (void*)b.sel, (void*)b.wt, (void*)b.p_first, (void*)b.wave_p,
                  (void*)b.deg_start, (void*)b.deg_off})
    if (q) (void)hipFree(q);
  b = DevBand();
}

template <typename T>
int upload_vec(const std::vector<T>& h, T** d) {
  *d = nullptr;
  const size_t n = h.empty() ? 1 : h.size();
  BH_HIP(hipMalloc((void**)d, n * sizeof(T)));
  if (!h.empty()) BH_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return BH_OK;
}

int check_L(int L) {
  if (L < 0 || L > BH_MAX_L) return set_error(BH_EINVAL, "bandlimit out of range");
  return BH_OK;
}

}  // namespace

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::clear() {
  for (auto& r : recs) {
    pool.push_back(r.start);
    pool.push_back(r.stop);
  }
  recs.clear();
}

void Profiler::destroy() {
  clear();
  for (hipEvent_t e : pool)
    if (e) (void)hipEventDestroy(e);
  pool.clear();
}

ProfScope::ProfScope(bh_plan* p, const std::string& name, hipStream_t s, int64_t work)
    : p_(p), s_(s) {
  if (!p_->prof.on) return;
  hipEvent_t a = p_->prof.take(), b = p_->prof.take();
  if (!a || !b || hipEventRecord(a, s_) != hipSuccess) {   // keep the events for later
    if (a) p_->prof.pool.push_back(a);
    if (b) p_->prof.pool.push_back(b);
    return;
  }
  p_->prof.recs.push_back({name, a, b, work});
  idx_ = (int)p_->prof.recs.size() - 1;
}

ProfScope::~ProfScope() {
  if (idx_ >= 0) (void)hipEventRecord(p_->prof.recs[idx_].stop, s_);
}

int grow(Buffer& b, size_t bytes) {
  if (bytes <= b.bytes) return BH_OK;
  if (b.ptr) {
    BH_HIP(hipDeviceSynchronize());
    BH_HIP(hipFree(b.ptr));
    b.ptr = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
    b.ptr = nullptr;
    (void)hipGetLastError();
    return set_error(BH_ENOMEM, "scratch allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return BH_OK;
}

int get_band(bh_plan* p, int L, const DevBand** out) {
  auto it = p->bands.find(L);
  if (it != p->bands.end()) {
    *out = &it->second;
    return BH_OK;
  }
  BandTables t = band_tables(L, p->L_max);
  t.rec.resize(t.rec.size() + 2 * kTablePad, 0.0);   // look-ahead padding
  DevBand d;
  d.L = L;
  d.n_classes = t.n_classes;
  d.n_entries = t.n_entries;
  d.n_deg = (int)t.deg_off.size();
  int rc;
  if ((rc = upload_vec(t.rec, &d.rec)) != BH_OK ||
      (rc = upload_vec(t.sel, &d.sel)) != BH_OK ||
      (rc = upload_vec(t.wt, &d.wt)) != BH_OK ||
      (rc = upload_vec(t.p_first, &d.p_first)) != BH_OK ||
      (rc = upload_vec(t.wave_p, &d.wave_p)) != BH_OK ||
      (rc = upload_vec(t.deg_start, &d.deg_start)) != BH_OK ||
      (rc = upload_vec(t.deg_off, &d.deg_off)) != BH_OK) {
    free_band(d);
    return rc;
  }
  p->bands[L] = d;
  *out = &p->bands[L];
  return BH_OK;
}

// BH_EINVAL (and the flag cleared) if a kernel of an earlier call on this
// plan met a template index outside its table or a volume row outside its
// stack.
int take_pending_error(bh_plan* p) {
  if (p->err_host && __atomic_exchange_n(p->err_host, 0, __ATOMIC_ACQ_REL) != 0)
    return set_error(BH_EINVAL,
                     "an earlier call on this plan had a template index outside "
                     "0..n_templates-1 or a volume row outside 0..n_vols-1; the results of "
                     "those particles are NaN");
  return BH_OK;
}

}  // namespace bh

using namespace bh;

// Coefficient arrays are read as (re, im) float pairs.
static bool pairs_aligned(const float* q) { return ((uintptr_t)q & 7u) == 0; }

extern "C" {

const char* bh_last_error(void) { return g_err.c_str(); }

int64_t bh_index_size(int L) {
  if (check_L(L) != BH_OK) return BH_EINVAL;
  try {
    return index_set(L).C;
  } catch (...) {
    return set_error(BH_ENOMEM, "host allocation failed");
  }
}

int bh_index_table(int L, int32_t* l, int32_t* k, int32_t* m, double* lambda) {
  return guarded([&]() -> int {
    int rc = check_L(L);
    if (rc != BH_OK) return rc;
    const IndexSet& s = index_set(L);
    for (const Radial& r : s.rad)
      for (int mm = -r.l; mm <= r.l; ++mm) {
        const int q = r.offset + r.l + mm;
        if (l) l[q] = r.l;
        if (k) k[q] = r.k;
        if (m) m[q] = mm;
        if (lambda) lambda[q] = r.lam;
      }
    return BH_OK;
  });
}

int bh_radial_count(int L) {
  return guarded([&]() -> int {
    int rc = check_L(L);
    if (rc != BH_OK) return rc;
    return (int)index_set(L).rad.size();
  });
}

int bh_radial_table(int L, int32_t* l, int32_t* k, double* lambda, double* c) {
  return guarded([&]() -> int {
    int rc = check_L(L);
    if (rc != BH_OK) return rc;
    const IndexSet& s = index_set(L);
    for (size_t i = 0; i < s.rad.size(); ++i) {
      if (l) l[i] = s.rad[i].l;
      if (k) k[i] = s.rad[i].k;
      if (lambda) lambda[i] = s.rad[i].lam;
      if (c) c[i] = s.rad[i].c;
    }
    return BH_OK;
  });
}

int64_t bh_ball_voxels(int N) {
  if (N < 1 || N > BH_MAX_N) return set_error(BH_EINVAL, "box edge out of range");
  try {
    return (int64_t)ball_voxels(N).size();
  } catch (...) {
    return set_error(BH_ENOMEM, "host allocation failed");
  }
}

int bh_plan_create(int N, int L_max, int device, bh_plan** out) {
  if (!out) return set_error(BH_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 2 || N > BH_MAX_N) return set_error(BH_EINVAL, "box edge out of range");
  if (L_max < 0 || L_max > BH_MAX_L) return set_error(BH_EINVAL, "bandlimit out of range");
  return guarded([&]() -> int {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
      return set_error(BH_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return set_error(BH_EINVAL, "device index out of range");
    DeviceGuard g(device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    int rc = noalloc_scratch_init(device);
    if (rc != BH_OK) return rc;
    // owned here until it is complete (an exception or error frees it)
    std::unique_ptr<bh_plan, void (*)(bh_plan*)> p(new bh_plan(), bh_plan_destroy);
    p->N = N;
    p->L_max = L_max;
    p->device = device;
    if (hipHostMalloc((void**)&p->err_host, sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      p->err_host = nullptr;
      (void)hipGetLastError();
      return set_error(BH_ENOMEM, "pinned error word allocation failed");
    }
    *p->err_host = 0;
    BH_HIP(hipHostGetDevicePointer((void**)&p->err_dev, p->err_host, 0));
    p->idx = &index_set(L_max);
    for (int L = 0; L <= L_max; ++L) p->band_size.push_back(index_set(L).C);
    rc = build_basis(p.get());
    if (rc != BH_OK) return rc;
    *out = p.release();
    return BH_OK;
  });
}

void bh_plan_destroy(bh_plan* p) {
  if (!p) return;
  DeviceGuard g(p->device);
  (void)hipDeviceSynchronize();
  for (void* q : {(void*)p->psi, (void*)p->psi_h, (void*)p->psi_l, (void*)p->vrep, (void*)p->csrc,
                  (void*)p->csgn})
    if (q) (void)hipFree(q);
  for (Buffer* b : {&p->gathered, &p->partial, &p->xi_scr, &p->state_scr, &p->misc_scr,
                    &p->prune_scr, &p->shift_scr, &p->newton_scr, &p->energy_scr, &p->xi_scr2,
                    &p->state_scr2, &p->misc_scr2})
    if (b->ptr) (void)hipFree(b->ptr);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->join_ev) (void)hipEventDestroy(p->join_ev);
  if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
  for (auto& kv : p->bands) free_band(kv.second);
  if (p->err_host) (void)hipHostFree(p->err_host);
  p->prof.destroy();
  delete p;
}

int bh_plan_check(bh_plan* p, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    BH_HIP(hipStreamSynchronize((hipStream_t)stream));
    return take_pending_error(p);
  });
}

int bh_plan_autotune(bh_plan* p, int64_t B, int n_restarts, const int32_t* bands, int n_bands,
                     int what, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 1 || B > (1LL << 16)) return set_error(BH_EINVAL, "tuning batch outside 1..65536");
  if (n_restarts < 1 || n_restarts > 1024) return set_error(BH_EINVAL, "bad restart count");
  if ((what & BH_TUNE_MARCH) && (n_bands < 1 || n_bands > 64 || !bands))
    return set_error(BH_EINVAL, "bad band list");
  if (what & BH_TUNE_MARCH)
    for (int i = 0; i < n_bands; ++i)
      if (bands[i] < 0 || bands[i] > p->L_max) return set_error(BH_EINVAL, "band outside 0..L_max");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    const hipStream_t s = (hipStream_t)stream;
    int rc = BH_OK;
    if ((what & BH_TUNE_MARCH) && (rc = tune_march(p, B, n_restarts, bands, n_bands, s)) != BH_OK)
      return rc;
    if ((what & BH_TUNE_EXPAND) && (rc = tune_expand_f32(p, B, s)) != BH_OK) return rc;
    if ((what & BH_TUNE_EXPAND_BF16) && (rc = tune_expand_bf16(p, B, s)) != BH_OK) return rc;
    BH_HIP(hipStreamSynchronize(s));
    return BH_OK;
  });
}

int bh_plan_set_tuning(bh_plan* p, int L, int waves, int persistent) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L < 0 || L > p->L_max) return set_error(BH_EINVAL, "L outside 0..L_max");
  if (waves != 0 && waves != 4 && waves != 5 && waves != 6 && waves != 8 && waves != 10 &&
      waves != 12 && waves != 16)
    return set_error(BH_EINVAL, "wave count must be 0 or one of 4, 5, 6, 8, 10, 12, 16");
  if (waves > 2 * L + 1 && waves > 4) return set_error(BH_EINVAL, "more waves than p-groups");
  p->tuned_waves[L] = waves;
  p->tuned_persist[L] = persistent ? 1 : 0;
  return BH_OK;
}

int bh_plan_tuning(const bh_plan* p, int L, int64_t B, int* waves, int* persistent,
                   int* split_f32, int* split_bf16) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L < 0 || L > p->L_max) return set_error(BH_EINVAL, "L outside 0..L_max");
  if (B < 1) return set_error(BH_EINVAL, "batch size out of range");
  if (waves) *waves = p->tuned_waves[L];
  if (persistent) *persistent = p->tuned_persist[L];
  DeviceGuard g(p->device);
  if (split_f32) *split_f32 = expand_split_f32(p, B, false);
  if (split_bf16) *split_bf16 = expand_split_bf16(p, B, false);
  return BH_OK;
}

int bh_profile_enable(bh_plan* p, int enable) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (enable) {
      BH_HIP(hipDeviceSynchronize());
      p->prof.clear();
    }
    p->prof.on = enable != 0;
    return BH_OK;
  });
}

int bh_profile_read(bh_plan* p, const char* name, int64_t* launches, double* total_ms,
                    int64_t* work) {
  if (!p || !name) return set_error(BH_EINVAL, "NULL argument");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    std::string pat(name);
    bool prefix = !pat.empty() && pat.back() == '*';
    if (prefix) pat.pop_back();
    int64_t n = 0, w = 0;
    double ms = 0.0;
    for (auto& r : p->prof.recs) {
      const bool hit = prefix ? r.name.compare(0, pat.size(), pat) == 0 : r.name == pat;
      if (!hit) continue;
      BH_HIP(hipEventSynchronize(r.stop));
      float t = 0.0f;
      BH_HIP(hipEventElapsedTime(&t, r.start, r.stop));
      ms += t;
      n += 1;
      w += r.work;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (work) *work = w;
    return BH_OK;
  });
}

int bh_plan_set_march_streams(bh_plan* p, int streams) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (streams != 1 && streams != 2) return set_error(BH_EINVAL, "march streams must be 1 or 2");
  p->march_streams = streams;
  return BH_OK;
}

int bh_profile_busy(bh_plan* p, const char* name, double* busy_ms) {
  if (!p || !name || !busy_ms) return set_error(BH_EINVAL, "NULL argument");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    std::string pat(name);
    bool prefix = !pat.empty() && pat.back() == '*';
    if (prefix) pat.pop_back();
    // [start, stop] of every matching launch, in ms from the first one recorded
    std::vector<std::pair<double, double>> iv;
    const Profiler::Rec* ref = nullptr;
    for (auto& r : p->prof.recs) {
      const bool hit = prefix ? r.name.compare(0, pat.size(), pat) == 0 : r.name == pat;
      if (!hit) continue;
      BH_HIP(hipEventSynchronize(r.stop));
      if (!ref) ref = &r;
      float t0 = 0.0f, t1 = 0.0f;
      BH_HIP(hipEventElapsedTime(&t0, ref->start, r.start));
      BH_HIP(hipEventElapsedTime(&t1, ref->start, r.stop));
      iv.push_back({(double)t0, (double)t1});
    }
    *busy_ms = interval_union(std::move(iv));
    return BH_OK;
  });
}

int64_t bh_plan_num_coeffs(const bh_plan* p, int L) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L < 0 || L > p->L_max) return set_error(BH_EINVAL, "L outside 0..L_max");
  return p->band_size[L];
}

int bh_expand(bh_plan* p, const float* vols, int64_t B, float* coeffs, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 0 || B > (1LL << 21)) return set_error(BH_EINVAL, "batch size out of range");
  if (B == 0) return BH_OK;
  if (!vols || !coeffs) return set_error(BH_EINVAL, "NULL buffer");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    return launch_expand(p, vols, B, coeffs, (hipStream_t)stream);
  });
}

int bh_expand_noalloc(bh_plan* p, const float* vols, int64_t B, float* coeffs, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 0 || B > (1LL << 21)) return set_error(BH_EINVAL, "batch size out of range");
  if (B == 0) return BH_OK;
  if (!vols || !coeffs) return set_error(BH_EINVAL, "NULL buffer");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    return launch_expand_noalloc(p, vols, B, coeffs, (hipStream_t)stream);
  });
}

int64_t bh_expand_noalloc_batch(const bh_plan* p) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  int64_t tiles = 0;
  noalloc_expand_pass(p, &tiles);
  return tiles * kGemmBM;
}

int bh_expand_ex(bh_plan* p, const float* vols, int64_t B, int mode, float* coeffs, float* coarse,
                 void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 0 || B > (1LL << 21)) return set_error(BH_EINVAL, "batch size out of range");
  const bool invariant = (mode & BH_EXPAND_BATCH_INVARIANT) != 0;
  mode &= ~BH_EXPAND_BATCH_INVARIANT;
  if (mode != BH_EXPAND_FP32 && mode != BH_EXPAND_BF16 && mode != BH_EXPAND_BF16X3)
    return set_error(BH_EINVAL, "unknown expansion mode");
  if (coarse && mode != BH_EXPAND_BF16X3)
    return set_error(BH_EINVAL, "a coarse output needs the BF16X3 mode");
  if (B == 0) return BH_OK;
  if (!vols || !coeffs) return set_error(BH_EINVAL, "NULL buffer");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    if (mode == BH_EXPAND_FP32)
      return launch_expand(p, vols, B, coeffs, (hipStream_t)stream, invariant);
    return launch_expand_bf16(p, vols, B, mode == BH_EXPAND_BF16X3, coeffs, coarse,
                              (hipStream_t)stream, invariant);
  });
}

int bh_expand_into(bh_plan* p, const float* vols, int64_t B, int mode, float* coeffs, int64_t ldc,
                   float* coarse, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 0 || B > (1LL << 21)) return set_error(BH_EINVAL, "batch size out of range");
  if (ldc < p->C || ldc > (1LL << 24)) return set_error(BH_EINVAL, "ldc smaller than C(L_max)");
  const bool invariant = (mode & BH_EXPAND_BATCH_INVARIANT) != 0;
  mode &= ~BH_EXPAND_BATCH_INVARIANT;
  if (mode != BH_EXPAND_FP32 && mode != BH_EXPAND_BF16 && mode != BH_EXPAND_BF16X3)
    return set_error(BH_EINVAL, "unknown expansion mode");
  if (coarse && mode != BH_EXPAND_BF16X3)
    return set_error(BH_EINVAL, "a coarse output needs the BF16X3 mode");
  if (B == 0) return BH_OK;
  if (!vols || !coeffs) return set_error(BH_EINVAL, "NULL buffer");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    if (mode == BH_EXPAND_FP32)
      return launch_expand(p, vols, B, coeffs, (hipStream_t)stream, invariant, nullptr, 1, ldc);
    return launch_expand_bf16(p, vols, B, mode == BH_EXPAND_BF16X3, coeffs, coarse,
                              (hipStream_t)stream, invariant, ldc);
  });
}

int bh_expand_rows(bh_plan* p, const float* vols, int64_t n_vols, const int64_t* rows, int64_t B,
                   int mode, float* coeffs, int64_t ldc, float* coarse, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 0 || B > (1LL << 21)) return set_error(BH_EINVAL, "batch size out of range");
  if (n_vols < 0 || n_vols > (1LL << 40) / ((int64_t)p->N * p->N * p->N))
    return set_error(BH_EINVAL, "volume count out of range");
  if (ldc == 0) ldc = p->C;
  if (ldc < p->C || ldc > (1LL << 24)) return set_error(BH_EINVAL, "ldc smaller than C(L_max)");
  const bool invariant = (mode & BH_EXPAND_BATCH_INVARIANT) != 0;
  mode &= ~BH_EXPAND_BATCH_INVARIANT;
  if (mode != BH_EXPAND_FP32 && mode != BH_EXPAND_BF16 && mode != BH_EXPAND_BF16X3)
    return set_error(BH_EINVAL, "unknown expansion mode");
  if (coarse && mode != BH_EXPAND_BF16X3)
    return set_error(BH_EINVAL, "a coarse output needs the BF16X3 mode");
  if (B == 0) return BH_OK;
  if (!vols || !rows || !coeffs) return set_error(BH_EINVAL, "NULL buffer");
  if (((uintptr_t)rows & 7u) != 0) return set_error(BH_EINVAL, "row table not 8-byte aligned");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    if (mode == BH_EXPAND_FP32)
      return launch_expand(p, vols, B, coeffs, (hipStream_t)stream, invariant, nullptr, 1, ldc,
                           rows, n_vols);
    return launch_expand_bf16(p, vols, B, mode == BH_EXPAND_BF16X3, coeffs, coarse,
                              (hipStream_t)stream, invariant, ldc, rows, n_vols);
  });
}

int bh_cross_power(bh_plan* p, const float* a, const float* b, int64_t B, int L, double* xi,
                   void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L < 0 || L > p->L_max) return set_error(BH_EINVAL, "L outside 0..L_max");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (B == 0) return BH_OK;
  if (!a || !b || !xi) return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(a) || !pairs_aligned(b))
    return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    const DevBand* band = nullptr;
    int rc = get_band(p, L, &band);
    if (rc != BH_OK) return rc;
    return launch_cross_power_dense(p, *band, a, b, B, xi, (hipStream_t)stream);
  });
}

static int correlate_common(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                            const double* euler, int R, double* score, double* grad, double* hess,
                            void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L < 0 || L > p->L_max) return set_error(BH_EINVAL, "L outside 0..L_max");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (R < 1 || R > (1 << 20)) return set_error(BH_EINVAL, "rotation count out of range");
  if (B == 0) return BH_OK;
  if (!a || !b || !euler || !score) return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(a) || !pairs_aligned(b))
    return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    const DevBand* band = nullptr;
    int rc = get_band(p, L, &band);
    if (rc != BH_OK) return rc;
    return launch_correlate(p, *band, a, b, B, euler, R, score, grad, hess, (hipStream_t)stream);
  });
}

int bh_correlate(bh_plan* p, const float* a, const float* b, int64_t B, int L, const double* euler,
                 int R, double* score, double* grad, void* stream) {
  return correlate_common(p, a, b, B, L, euler, R, score, grad, nullptr, stream);
}

int bh_correlate_hess(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                      const double* euler, int R, double* score, double* grad, double* hess,
                      void* stream) {
  if (!hess) return set_error(BH_EINVAL, "NULL buffer");
  return correlate_common(p, a, b, B, L, euler, R, score, grad, hess, stream);
}

int bh_degree_energy(bh_plan* p, const float* a, const float* b, int64_t B, int L,
                     double* energy, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L < 0 || L > p->L_max) return set_error(BH_EINVAL, "L outside 0..L_max");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (B == 0) return BH_OK;
  if (!a || !b || !energy) return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(a) || !pairs_aligned(b))
    return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    const DevBand* band = nullptr;
    int rc = get_band(p, L, &band);
    if (rc != BH_OK) return rc;
    return launch_degree_energy(p, *band, a, b, nullptr, 1, B, energy, (hipStream_t)stream);
  });
}

int bh_select_bands(bh_plan* p, const float* a, const float* templates, int n_templates,
                    const int32_t* tmpl_idx, int64_t B, int L_top, const double* thresholds,
                    int n_tau, int32_t* bands, int32_t* common, double* ratio, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (L_top < 0 || L_top > p->L_max) return set_error(BH_EINVAL, "L_top outside 0..L_max");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (n_templates < 1 || n_templates > (1 << 20)) return set_error(BH_EINVAL, "bad template count");
  if (n_templates > 1 && !tmpl_idx) return set_error(BH_EINVAL, "template index table is NULL");
  if (n_tau < 1 || n_tau > kMaxBandThresholds || !thresholds)
    return set_error(BH_EINVAL, "threshold count outside 1..16");
  BandThresholds th = {};
  for (int j = 0; j < n_tau; ++j) {
    if (!(thresholds[j] >= 0.0 && thresholds[j] <= 1.0))
      return set_error(BH_EINVAL, "thresholds must lie in [0, 1]");
    th.t[j] = thresholds[j];
  }
  int rc = take_pending_error(p);
  if (rc != BH_OK) return rc;
  if (B == 0) return BH_OK;
  if (!a || !templates || !bands) return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(a) || !pairs_aligned(templates))
    return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    const DevBand* band = nullptr;
    int rc2 = get_band(p, L_top, &band);
    if (rc2 != BH_OK) return rc2;
    return launch_select_bands(p, *band, a, templates, n_templates > 1 ? tmpl_idx : nullptr,
                               n_templates, B, th, n_tau, bands, common, ratio,
                               (hipStream_t)stream);
  });
}

static int check_align_opts(const bh_plan* p, const bh_align_opts* o) {
  if (o->n_bands < 1 || o->n_bands > 16 || !o->bands) return set_error(BH_EINVAL, "bad band list");
  for (int i = 0; i < o->n_bands; ++i)
    if (o->bands[i] < 0 || o->bands[i] > p->L_max) return set_error(BH_EINVAL, "band outside 0..L_max");
  if (o->steps_per_band < 0 || o->steps_per_band > 10000) return set_error(BH_EINVAL, "bad step count");
  if (o->n_restarts < 1 || o->n_restarts > 65536) return set_error(BH_EINVAL, "bad restart count");
  if (!(o->step_init > 0) || !(o->step_grow > 0) || !(o->step_shrink > 0))
    return set_error(BH_EINVAL, "step parameters must be positive");
  if (o->newton_bands < 0 || o->newton_bands > o->n_bands)
    return set_error(BH_EINVAL, "newton_bands outside 0..n_bands");
  if (o->newton_steps < 0 || o->newton_steps > 10000) return set_error(BH_EINVAL, "bad Newton step count");
  if (o->n_keep < 0 || o->n_keep > 64) return set_error(BH_EINVAL, "n_keep outside 0..64");
  if (o->n_keep > 0 && o->n_keep < o->n_restarts && o->n_restarts > kPruneMaxP)
    return set_error(BH_EUNSUPPORTED, "candidate pruning needs n_restarts <= 1024");
  if (!(o->keep_min_sep >= 0.0) || o->keep_min_sep > 3.141592653589793)
    return set_error(BH_EINVAL, "keep_min_sep outside [0, pi]");
  return BH_OK;
}

int bh_align_t(bh_plan* p, const float* a, const float* templates, int n_templates,
               const int32_t* tmpl_idx, int64_t B, const bh_align_opts* o, const double* starts,
               double* euler_out, double* score_out, double* all_euler, double* all_score,
               void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (!o) return set_error(BH_EINVAL, "opts is NULL");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (n_templates < 1 || n_templates > (1 << 20)) return set_error(BH_EINVAL, "bad template count");
  if (n_templates > 1 && !tmpl_idx) return set_error(BH_EINVAL, "template index table is NULL");
  int rc = check_align_opts(p, o);
  if (rc != BH_OK) return rc;
  if ((rc = take_pending_error(p)) != BH_OK) return rc;
  if (B == 0) return BH_OK;
  if (!a || !templates || !starts || !euler_out || !score_out) return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(a) || !pairs_aligned(templates))
    return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    return launch_align(p, a, templates, n_templates > 1 ? tmpl_idx : nullptr, n_templates, B, *o,
                        starts, euler_out, score_out, all_euler, all_score, (hipStream_t)stream);
  });
}

int bh_align_shifts(bh_plan* p, const float* vols, int64_t B, const int32_t* shifts, int S,
                    const float* b, const bh_align_opts* o, const double* starts,
                    double* euler_out, double* score_out, int32_t* shift_out, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (!o) return set_error(BH_EINVAL, "opts is NULL");
  if (S < 1 || S > kMaxShifts) return set_error(BH_EINVAL, "shift count outside 1..125");
  if (!shifts) return set_error(BH_EINVAL, "shift table is NULL");
  for (int i = 0; i < 3 * S; ++i)
    if (shifts[i] < -p->N || shifts[i] > p->N) return set_error(BH_EINVAL, "shift beyond the box");
  if (B < 0 || B * (int64_t)S > (1LL << 21)) return set_error(BH_EINVAL, "batch size out of range");
  if (B == 0) return BH_OK;
  if (!vols || !b || !starts || !euler_out || !score_out || !shift_out)
    return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(b)) return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  int rc = check_align_opts(p, o);
  if (rc != BH_OK) return rc;
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    return launch_align_shifts(p, vols, B, shifts, S, b, *o, starts, euler_out, score_out,
                               shift_out, (hipStream_t)stream);
  });
}

int bh_align_uneven(bh_plan* p, const float* a, int64_t lda, const int32_t* Lp,
                    const float* templates, int64_t ldt, int n_templates, const int32_t* tmpl_idx,
                    int64_t B, const bh_align_opts* o, const double* starts, double* euler_out,
                    double* score_out, double* all_euler, double* all_score, void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (!o) return set_error(BH_EINVAL, "opts is NULL");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (n_templates < 1 || n_templates > (1 << 20)) return set_error(BH_EINVAL, "bad template count");
  if (n_templates > 1 && !tmpl_idx) return set_error(BH_EINVAL, "template index table is NULL");
  int rc = check_align_opts(p, o);
  if (rc != BH_OK) return rc;
  if ((rc = take_pending_error(p)) != BH_OK) return rc;
  if (B == 0) return BH_OK;
  if (!a || !Lp || !templates || !starts || !euler_out || !score_out)
    return set_error(BH_EINVAL, "NULL buffer");
  if (!pairs_aligned(a) || !pairs_aligned(templates))
    return set_error(BH_EINVAL, "coefficient buffer not 8-byte aligned");
  for (int i = 1; i < o->n_bands; ++i)
    if (o->bands[i] <= o->bands[i - 1]) return set_error(BH_EINVAL, "bands must increase");
  for (int64_t i = 1; i < B; ++i)
    if (Lp[i] > Lp[i - 1]) return set_error(BH_EINVAL, "bandlimits must not increase along the batch");
  if (Lp[B - 1] < o->bands[0]) return set_error(BH_EINVAL, "every particle must take the first band");
  std::vector<int64_t> active(o->n_bands, 0);
  int top = 0;                          // largest band any particle takes
  for (int i = 0; i < o->n_bands; ++i) {
    int64_t n = 0;
    while (n < B && Lp[n] >= o->bands[i]) ++n;
    active[i] = n;
    if (n > 0) top = o->bands[i];
  }
  const int64_t need = p->band_size[top];
  if (lda < need || ldt < need) return set_error(BH_EINVAL, "row stride below the largest band's C(L)");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    return launch_align(p, a, templates, n_templates > 1 ? tmpl_idx : nullptr, n_templates, B, *o,
                        starts, euler_out, score_out, all_euler, all_score, (hipStream_t)stream,
                        lda, ldt, active.data());
  });
}

int bh_prune_candidates(bh_plan* p, const double* euler, const double* score, int64_t B, int P,
                        int K, double min_sep, double* euler_out, double* score_out,
                        void* stream) {
  if (!p) return set_error(BH_EINVAL, "plan is NULL");
  if (B < 0 || B > (1LL << 24)) return set_error(BH_EINVAL, "batch size out of range");
  if (P < 1 || P > kPruneMaxP) return set_error(BH_EINVAL, "restart count outside 1..1024");
  if (K < 1 || K > 64 || K > P) return set_error(BH_EINVAL, "K outside 1..min(64, P)");
  if (!(min_sep >= 0.0) || min_sep > 3.141592653589793)
    return set_error(BH_EINVAL, "min_sep outside [0, pi]");
  if (B == 0) return BH_OK;
  if (!euler || !score || !euler_out || !score_out) return set_error(BH_EINVAL, "NULL buffer");
  return guarded([&]() -> int {
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(BH_EDEVICE, "hipSetDevice failed");
    return launch_prune(p, euler, score, B, P, K, min_sep, euler_out, score_out,
                        (hipStream_t)stream);
  });
}

int bh_align(bh_plan* p, const float* a, const float* b, int64_t B, const bh_align_opts* o,
             const double* starts, double* euler_out, double* score_out, double* all_euler,
             double* all_score, void* stream) {
  return bh_align_t(p, a, b, 1, nullptr, B, o, starts, euler_out, score_out, all_euler, all_score,
                    stream);
}

}  // extern "C"
