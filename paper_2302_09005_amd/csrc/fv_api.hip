// C ABI of libfv (declared and documented in include/fv.h): host-side
// argument validation, dispatch to the kernel launchers, error reporting.
// Nothing here allocates device memory, copies to the host or synchronises.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>

#include "fv_internal.hpp"

namespace {

thread_local char g_err[512] = "";
thread_local fvk::LaunchEvents g_events;

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = '\0';
  return FV_OK;
}

int64_t ipow64(int64_t b, int e) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}

int check_shape(int dim, int p, int halo, int s) {
  if (dim != 2 && dim != 3) return fail(FV_EINVAL, "dim must be 2 or 3 (got %d)", dim);
  if (halo != 1) return fail(FV_EINVAL, "halo width must be 1 (got %d)", halo);
  if (s != dim + 2) return fail(FV_EINVAL, "s must be dim + 2 = %d (got %d)", dim + 2, s);
  if (p < 1) return fail(FV_EINVAL, "p must be positive (got %d)", p);
  if (!fvk::update_supported(dim, p))
    return fail(FV_EUNSUPPORTED, "no kernel instance for dim=%d p=%d", dim, p);
  return FV_OK;
}

int launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FV_EHIP, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

}  // namespace

namespace fvk {
LaunchEvents& launch_events() { return g_events; }

int device_cu_count() {
  static std::atomic<int> cu_count[64];
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  cus = cu_count[dev].load(std::memory_order_relaxed);
  if (cus == 0 &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
    cu_count[dev].store(cus, std::memory_order_relaxed);
  return cus;
}
}  // namespace fvk

extern "C" {

int fv_set_launch_events(void* start_event, void* stop_event) {
  if ((start_event == nullptr) != (stop_event == nullptr))
    return fail(FV_EINVAL, "give both events or neither");
  g_events.start = (hipEvent_t)start_event;
  g_events.stop = (hipEvent_t)stop_event;
  return ok();
}


const char* fv_last_error(void) { return g_err; }

int fv_abi_version(void) { return 1; }

int fv_supported(int dim, int p) { return fvk::update_supported(dim, p) ? 1 : 0; }

int fv_check_patches(const fv_patch* host_patches, int64_t n, int dim, int p, int q_in_halo,
                     int q_out_halo, int64_t q_in_len, int64_t q_out_len) {
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (n > 0 && !host_patches) return fail(FV_EINVAL, "patches is NULL");
  if (dim != 2 && dim != 3) return fail(FV_EINVAL, "dim must be 2 or 3");
  if (p < 1) return fail(FV_EINVAL, "p must be positive");
  const int s = dim + 2;
  const int64_t blk_in = s * (q_in_halo ? ipow64(p + 2, dim) : ipow64(p, dim));
  const int64_t blk_out = s * (q_out_halo ? ipow64(p + 2, dim) : ipow64(p, dim));
  for (int64_t b = 0; b < n; ++b) {
    const fv_patch& d = host_patches[b];
    if (d.p != p) return fail(FV_EINVAL, "patch %lld: p=%d, call p=%d", (long long)b, d.p, p);
    if (d.q_in < 0 || d.q_in > q_in_len - blk_in)
      return fail(FV_EINVAL, "patch %lld: input block outside q_in", (long long)b);
    if (d.q_out < 0 || d.q_out > q_out_len - blk_out)
      return fail(FV_EINVAL, "patch %lld: output block outside q_out", (long long)b);
    for (int j = 0; j < dim; ++j)
      if (!(d.dx[j] > 0.0) || !isfinite(d.dx[j]))
        return fail(FV_EINVAL, "patch %lld: dx[%d] must be finite and > 0", (long long)b, j);
    if (!(d.dt >= 0.0) || !isfinite(d.dt))
      return fail(FV_EINVAL, "patch %lld: dt must be finite and >= 0", (long long)b);
  }
  // output blocks must be pairwise disjoint: sort a copy of the offsets and
  // compare neighbours
  if (n > 1) {
    int64_t* offs = new (std::nothrow) int64_t[n];
    if (!offs) return fail(FV_EINVAL, "out of host memory while checking overlaps");
    for (int64_t b = 0; b < n; ++b) offs[b] = host_patches[b].q_out;
    std::sort(offs, offs + n);
    int64_t bad = -1;
    for (int64_t b = 1; b < n && bad < 0; ++b)
      if (offs[b] - offs[b - 1] < blk_out) bad = b;
    delete[] offs;
    if (bad >= 0) return fail(FV_EINVAL, "output blocks overlap");
  }
  return ok();
}

}  // extern "C"

namespace {

template <typename T>
int overlap_check(const T* q_in, int64_t q_in_len, const T* q_out, int64_t q_out_len) {
  const char* a0 = (const char*)q_in;
  const char* a1 = a0 + q_in_len * (int64_t)sizeof(T);
  const char* b0 = (const char*)q_out;
  const char* b1 = b0 + q_out_len * (int64_t)sizeof(T);
  if (a0 < b1 && b0 < a1) return fail(FV_EINVAL, "q_in and q_out overlap");
  return FV_OK;
}

template <typename T>
int batch_update_impl(const char* name, const fv_patch* patches, int64_t n, const T* q_in,
                      int64_t q_in_len, T* q_out, int64_t q_out_len, int q_out_halo, int dim,
                      int p, int halo, int s, double gamma, const double* dt_dev, double* max_eig,
                      void* stream) {
  int rc = check_shape(dim, p, halo, s);
  if (rc) return rc;
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (q_out_halo != 0 && q_out_halo != 1) return fail(FV_EINVAL, "q_out_halo must be 0 or 1");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (n == 0) return ok();
  if (!patches || !q_in || !q_out) return fail(FV_EINVAL, "null device pointer");
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  if ((rc = overlap_check(q_in, q_in_len, q_out, q_out_len))) return rc;
  rc = fvk::launch_update<T>(patches, n, q_in, q_in_len, q_out, q_out_len, q_out_halo, dim, p,
                             gamma, dt_dev, max_eig, (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched(name);
}

template <typename T>
int batch_update_gather_impl(const char* name, const fv_patch* patches, int64_t n,
                             const int64_t* neighbours, const T* q_in, int64_t q_in_len,
                             T* q_out, int64_t q_out_len, int q_out_halo, int dim, int p, int s,
                             double gamma, const double* dt_dev, double* max_eig, void* stream) {
  int rc = check_shape(dim, p, 1, s);
  if (rc) return rc;
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (q_out_halo != 0 && q_out_halo != 1) return fail(FV_EINVAL, "q_out_halo must be 0 or 1");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (n == 0) return ok();
  if (!patches || !neighbours || !q_in || !q_out) return fail(FV_EINVAL, "null device pointer");
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  if ((rc = overlap_check(q_in, q_in_len, q_out, q_out_len))) return rc;
  rc = fvk::launch_update_gather<T>(patches, n, neighbours, q_in, q_in_len, q_out, q_out_len,
                                    q_out_halo, dim, p, gamma, dt_dev, max_eig,
                                    (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched(name);
}

template <typename T>
int step_gather_impl(const char* name, const fv_patch* patches, int64_t n,
                     const int64_t* neighbours, const T* q_in, int64_t q_in_len, T* q_out,
                     int64_t q_out_len, int dim, int p, int s, double gamma, double cfl,
                     const double* dt_dev, double* max_eig, double* dt_next, double* lambda_out,
                     uint64_t* workspace, int64_t workspace_words, void* stream) {
  int rc = check_shape(dim, p, 1, s);
  if (rc) return rc;
  if (n < 1) return fail(FV_EINVAL, "n_patches must be >= 1");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(FV_EINVAL, "cfl must be finite and > 0");
  if (!patches || !neighbours || !q_in || !q_out || !dt_dev || !dt_next || !workspace)
    return fail(FV_EINVAL, "null device pointer");
  if (dt_next == dt_dev) return fail(FV_EINVAL, "dt_next must not alias dt_dev");
  const int64_t need = fvk::step_workspace_words(fvk::update_workgroups(dim, p, n));
  if (workspace_words < need) return fail(FV_EINVAL, "workspace needs %lld words", (long long)need);
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  if ((rc = overlap_check(q_in, q_in_len, q_out, q_out_len))) return rc;
  fvk::CflOut co;
  co.cfl = cfl;
  co.dt_next = dt_next;
  co.lambda_out = lambda_out;
  co.ws = reinterpret_cast<unsigned long long*>(workspace);
  rc = fvk::launch_step_gather<T>(patches, n, neighbours, q_in, q_in_len, q_out, q_out_len, dim,
                                  p, gamma, dt_dev, max_eig, co, (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched(name);
}

template <typename T>
int step_pipelined_impl(const char* name, const fv_patch* patches, int64_t n,
                        const int64_t* neighbours, const T* q_in, int64_t q_in_len, T* q_out,
                        int64_t q_out_len, int dim, int p, int s, double gamma, double cfl,
                        int phase, const double* dt_in, double* dt_used, double* max_eig,
                        double* lambda_out, uint64_t* workspace, int64_t workspace_words,
                        void* stream) {
  int rc = check_shape(dim, p, 1, s);
  if (rc) return rc;
  if (n < 1) return fail(FV_EINVAL, "n_patches must be >= 1");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(FV_EINVAL, "cfl must be finite and > 0");
  if (phase < 0 || phase > 2) return fail(FV_EINVAL, "phase must be 0, 1 or 2");
  if (!patches || !neighbours || !q_in || !q_out || !workspace)
    return fail(FV_EINVAL, "null device pointer");
  const int64_t need = fvk::pipelined_workspace_words();
  if (workspace_words < need) return fail(FV_EINVAL, "workspace needs %lld words", (long long)need);
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  if ((rc = overlap_check(q_in, q_in_len, q_out, q_out_len))) return rc;
  fvk::CflOut co;
  co.cfl = cfl;
  co.lambda_out = lambda_out;
  co.ws = reinterpret_cast<unsigned long long*>(workspace);
  co.phase = phase;
  co.dt_in = dt_in;
  co.dt_used = dt_used;
  rc = fvk::launch_step_pipelined<T>(patches, n, neighbours, q_in, q_in_len, q_out, q_out_len,
                                     dim, p, gamma, max_eig, co, (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched(name);
}

template <typename T>
int max_eigenvalue_impl(const char* name, const fv_patch* patches, int64_t n, const T* q,
                        int64_t q_len, int q_halo, int which, int dim, int p, int s, double gamma,
                        double* per_patch, double* global, void* stream) {
  int rc = check_shape(dim, p, 1, s);
  if (rc) return rc;
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (q_halo != 0 && q_halo != 1) return fail(FV_EINVAL, "q_halo must be 0 or 1");
  if (which != FV_OFFSETS_IN && which != FV_OFFSETS_OUT)
    return fail(FV_EINVAL, "which_offsets must be FV_OFFSETS_IN or FV_OFFSETS_OUT");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (n == 0) {
    if (!global) return ok();
    // nothing to reduce: the reduction kernel writes the documented 0
    fvk::launch_reduce_cfl(patches, 0, per_patch, dim, 1.0, global, nullptr, (hipStream_t)stream);
    return launched(name);
  }
  if (!patches || !q || !per_patch) return fail(FV_EINVAL, "null device pointer");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  rc = fvk::launch_patch_max<T>(patches, n, q, q_len, q_halo, which, dim, p, gamma, per_patch,
                                (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  if (global)
    fvk::launch_reduce_cfl(patches, n, per_patch, dim, 1.0, global, nullptr, (hipStream_t)stream);
  return launched(name);
}

template <typename T>
int totals_impl(const char* name, const fv_patch* patches, int64_t n, const T* q, int64_t q_len,
                int q_halo, int which, int dim, int p, int s, double* per_patch, double* totals,
                void* stream) {
  int rc = check_shape(dim, p, 1, s);
  if (rc) return rc;
  if (n < 1) return fail(FV_EINVAL, "n_patches must be >= 1");
  if (q_halo != 0 && q_halo != 1) return fail(FV_EINVAL, "q_halo must be 0 or 1");
  if (which != FV_OFFSETS_IN && which != FV_OFFSETS_OUT)
    return fail(FV_EINVAL, "which_offsets must be FV_OFFSETS_IN or FV_OFFSETS_OUT");
  if (!patches || !q || !per_patch) return fail(FV_EINVAL, "null device pointer");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  rc = fvk::launch_totals<T>(patches, n, q, q_len, q_halo, which, dim, p, per_patch, totals,
                             (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched(name);
}

template <typename T>
int step_local_impl(const char* name, fv_patch* patches, int64_t n, const int64_t* neighbours,
                    const fv_mixed_plan* plan, const T* q_in, int64_t q_in_len, T* q_out,
                    int64_t q_out_len, int dim, int s, double gamma, double cfl,
                    double* max_eig, int schedule, int grid, void* stream) {
  if (dim != 3) return fail(FV_EUNSUPPORTED, "uneven batches are 3-D only (got dim=%d)", dim);
  if (s != dim + 2) return fail(FV_EINVAL, "s must be dim + 2 = %d (got %d)", dim + 2, s);
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(FV_EINVAL, "cfl must be finite and > 0");
  if (schedule != FV_SCHED_PER_SIZE && schedule != FV_SCHED_PERSISTENT &&
      schedule != FV_SCHED_PATCHWISE)
    return fail(FV_EINVAL, "schedule must be one of FV_SCHED_PER_SIZE, FV_SCHED_PERSISTENT, "
                           "FV_SCHED_PATCHWISE (got %d)", schedule);
  if (grid < 0) return fail(FV_EINVAL, "persistent_workgroups < 0");
  if (!plan) return fail(FV_EINVAL, "null plan");
  if (n == 0) return ok();
  if (!patches || !neighbours || !q_in || !q_out || !plan->order || !plan->units)
    return fail(FV_EINVAL, "null device pointer");
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  int64_t next = 0, units = 0;
  for (int c = 0; c < 3; ++c) {
    const int64_t cnt = plan->class_count[c];
    if (cnt == 0) continue;
    const int pp = plan->class_p[c];
    const int ppu = fvk::mixed_patches_per_unit(pp);
    if (ppu == 0) return fail(FV_EUNSUPPORTED, "plan class %d: no instance for p=%d", c, pp);
    if (cnt < 0 || plan->class_first[c] != next)
      return fail(FV_EINVAL, "plan class %d does not continue the order at %lld", c,
                  (long long)next);
    next += cnt;
    units += (cnt + ppu - 1) / ppu;
  }
  if (next != n) return fail(FV_EINVAL, "plan covers %lld patches, batch has %lld",
                             (long long)next, (long long)n);
  if (plan->n_units != units)
    return fail(FV_EINVAL, "plan has %lld work units, its classes need %lld",
                (long long)plan->n_units, (long long)units);
  int rc = overlap_check(q_in, q_in_len, q_out, q_out_len);
  if (rc) return rc;
  rc = fvk::launch_step_local<T>(patches, n, neighbours, *plan, q_in, q_in_len, q_out, q_out_len,
                                 gamma, cfl, max_eig, schedule, grid, (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance in the plan");
  return launched(name);
}

}  // namespace

extern "C" {

int fv_plan_mixed(const fv_patch* host_patches, int64_t n, int dim, int64_t* order,
                  fv_work_unit* units, fv_mixed_plan* plan) {
  if (dim != 3) return fail(FV_EUNSUPPORTED, "uneven batches are 3-D only (got dim=%d)", dim);
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (!plan) return fail(FV_EINVAL, "null plan");
  if (n > 0 && (!host_patches || !order || !units)) return fail(FV_EINVAL, "null host pointer");
  static const int sizes[3] = {16, 8, 4};  // biggest units first
  int64_t count[3] = {0, 0, 0};
  for (int64_t b = 0; b < n; ++b) {
    const int pp = host_patches[b].p;
    int c = 0;
    while (c < 3 && sizes[c] != pp) ++c;
    if (c == 3) return fail(FV_EUNSUPPORTED, "patch %lld: p=%d not in {4, 8, 16}",
                            (long long)b, pp);
    ++count[c];
  }
  int64_t pos[3];
  int64_t first = 0, nu = 0;
  for (int c = 0; c < 3; ++c) {
    plan->class_p[c] = sizes[c];
    plan->class_first[c] = first;
    plan->class_count[c] = count[c];
    pos[c] = first;
    first += count[c];
  }
  for (int64_t b = 0; b < n; ++b) {  // stable counting sort by size class
    const int pp = host_patches[b].p;
    const int c = pp == 16 ? 0 : pp == 8 ? 1 : 2;
    order[pos[c]++] = b;
  }
  for (int c = 0; c < 3; ++c) {
    const int ppu = fvk::mixed_patches_per_unit(sizes[c]);
    for (int64_t k = 0; k < count[c]; k += ppu) {
      units[nu].p = sizes[c];
      units[nu].count = (int32_t)std::min<int64_t>(ppu, count[c] - k);
      units[nu].first = plan->class_first[c] + k;
      ++nu;
    }
  }
  plan->order = nullptr;
  plan->units = nullptr;
  plan->n_units = nu;
  return ok();
}

int fv_step_local(fv_patch* patches, int64_t n, const int64_t* neighbours,
                  const fv_mixed_plan* plan, const double* q_in, int64_t q_in_len, double* q_out,
                  int64_t q_out_len, int dim, int s, double gamma, double cfl, double* max_eig,
                  int schedule, int persistent_workgroups, void* stream) {
  return step_local_impl<double>("fv_step_local", patches, n, neighbours, plan, q_in, q_in_len,
                                 q_out, q_out_len, dim, s, gamma, cfl, max_eig, schedule,
                                 persistent_workgroups, stream);
}

int fv_step_local_f32(fv_patch* patches, int64_t n, const int64_t* neighbours,
                      const fv_mixed_plan* plan, const float* q_in, int64_t q_in_len,
                      float* q_out, int64_t q_out_len, int dim, int s, double gamma, double cfl,
                      double* max_eig, int schedule, int persistent_workgroups, void* stream) {
  return step_local_impl<float>("fv_step_local_f32", patches, n, neighbours, plan, q_in,
                                q_in_len, q_out, q_out_len, dim, s, gamma, cfl, max_eig,
                                schedule, persistent_workgroups, stream);
}

int fv_local_timestep(fv_patch* patches, int64_t n, const double* per_patch, int dim, double cfl,
                      void* stream) {
  if (dim != 2 && dim != 3) return fail(FV_EINVAL, "dim must be 2 or 3");
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(FV_EINVAL, "cfl must be finite and > 0");
  if (n == 0) return ok();
  if (!patches || !per_patch) return fail(FV_EINVAL, "null device pointer");
  fvk::launch_local_dt(patches, n, per_patch, dim, cfl, (hipStream_t)stream);
  return launched("fv_local_timestep");
}

}  // extern "C"

namespace {

}  // namespace

extern "C" {

int fv_batch_update(const fv_patch* patches, int64_t n, const double* q_in, int64_t q_in_len,
                    double* q_out, int64_t q_out_len, int q_out_halo, int dim, int p, int halo,
                    int s, double gamma, const double* dt_dev, double* max_eig, void* stream) {
  return batch_update_impl("fv_batch_update", patches, n, q_in, q_in_len, q_out, q_out_len,
                           q_out_halo, dim, p, halo, s, gamma, dt_dev, max_eig, stream);
}

int fv_batch_update_f32(const fv_patch* patches, int64_t n, const float* q_in, int64_t q_in_len,
                        float* q_out, int64_t q_out_len, int q_out_halo, int dim, int p, int halo,
                        int s, double gamma, const double* dt_dev, double* max_eig,
                        void* stream) {
  return batch_update_impl("fv_batch_update_f32", patches, n, q_in, q_in_len, q_out, q_out_len,
                           q_out_halo, dim, p, halo, s, gamma, dt_dev, max_eig, stream);
}

int fv_batch_update_gather(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                           const double* q_in, int64_t q_in_len, double* q_out,
                           int64_t q_out_len, int q_out_halo, int dim, int p, int s,
                           double gamma, const double* dt_dev, double* max_eig, void* stream) {
  return batch_update_gather_impl("fv_batch_update_gather", patches, n, neighbours, q_in,
                                  q_in_len, q_out, q_out_len, q_out_halo, dim, p, s, gamma,
                                  dt_dev, max_eig, stream);
}

int fv_batch_update_gather_f32(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                               const float* q_in, int64_t q_in_len, float* q_out,
                               int64_t q_out_len, int q_out_halo, int dim, int p, int s,
                               double gamma, const double* dt_dev, double* max_eig,
                               void* stream) {
  return batch_update_gather_impl("fv_batch_update_gather_f32", patches, n, neighbours, q_in,
                                  q_in_len, q_out, q_out_len, q_out_halo, dim, p, s, gamma,
                                  dt_dev, max_eig, stream);
}

int64_t fv_step_workspace_words(int64_t n, int dim, int p) {
  if (n < 1 || !fvk::update_supported(dim, p)) return 0;
  return fvk::step_workspace_words(fvk::update_workgroups(dim, p, n));
}

int fv_step_gather(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                   const double* q_in, int64_t q_in_len, double* q_out, int64_t q_out_len,
                   int dim, int p, int s, double gamma, double cfl, const double* dt_dev,
                   double* max_eig, double* dt_next, double* lambda_out, uint64_t* workspace,
                   int64_t workspace_words, void* stream) {
  return step_gather_impl("fv_step_gather", patches, n, neighbours, q_in, q_in_len, q_out,
                          q_out_len, dim, p, s, gamma, cfl, dt_dev, max_eig, dt_next, lambda_out,
                          workspace, workspace_words, stream);
}

int64_t fv_step_pipelined_workspace_words(int64_t n, int dim, int p) {
  if (n < 1 || !fvk::update_supported(dim, p)) return 0;
  return fvk::pipelined_workspace_words();
}

int fv_step_gather_pipelined(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                             const double* q_in, int64_t q_in_len, double* q_out,
                             int64_t q_out_len, int dim, int p, int s, double gamma, double cfl,
                             int phase, const double* dt_in, double* dt_used, double* max_eig,
                             double* lambda_out, uint64_t* workspace, int64_t workspace_words,
                             void* stream) {
  return step_pipelined_impl("fv_step_gather_pipelined", patches, n, neighbours, q_in, q_in_len,
                             q_out, q_out_len, dim, p, s, gamma, cfl, phase, dt_in, dt_used,
                             max_eig, lambda_out, workspace, workspace_words, stream);
}

int fv_step_gather_pipelined_f32(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                                 const float* q_in, int64_t q_in_len, float* q_out,
                                 int64_t q_out_len, int dim, int p, int s, double gamma,
                                 double cfl, int phase, const double* dt_in, double* dt_used,
                                 double* max_eig, double* lambda_out, uint64_t* workspace,
                                 int64_t workspace_words, void* stream) {
  return step_pipelined_impl("fv_step_gather_pipelined_f32", patches, n, neighbours, q_in,
                             q_in_len, q_out, q_out_len, dim, p, s, gamma, cfl, phase, dt_in,
                             dt_used, max_eig, lambda_out, workspace, workspace_words, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// fv_step_gather without a workspace argument: the fused CFL tree's slots live
// in a static device array.  Host code never passes the array's name to a
// kernel (in host code it names a host-side stand-in); it looks up the array's
// device address once per device and passes that.
// ---------------------------------------------------------------------------
namespace {

static __device__ __align__(256) unsigned long long scratch[FV_NOALLOC_SCRATCH_WORDS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

__global__ void clear_words_kernel(unsigned long long* w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0ull;
}

// Device address of this device's scratch array; on the first call for the
// device it is looked up and cleared (a kernel on `st`, ordered before the
// caller's launch).  nullptr on a HIP error (message in g_err).
unsigned long long* device_scratch(hipStream_t st) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    fail(FV_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    fail(FV_EHIP, "device index %d out of range", dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    fail(FV_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    return nullptr;
  }
  unsigned long long* w = static_cast<unsigned long long*>(ptr);
  hipLaunchKernelGGL(clear_words_kernel, dim3(64), dim3(256), 0, st, w,
                     (int64_t)FV_NOALLOC_SCRATCH_WORDS);
  e = hipGetLastError();
  if (e != hipSuccess) {
    fail(FV_EHIP, "clearing the scratch array: %s", hipGetErrorString(e));
    return nullptr;
  }
  g_scratch_ptr[dev] = w;
  return w;
}

}  // namespace

extern "C" {

int fv_step_gather_noalloc(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                           const double* q_in, int64_t q_in_len, double* q_out,
                           int64_t q_out_len, int dim, int p, int s, double gamma, double cfl,
                           const double* dt_dev, double* max_eig, double* dt_next,
                           double* lambda_out, void* stream) {
  int rc = check_shape(dim, p, 1, s);
  if (rc) return rc;
  if (n < 1) return fail(FV_EINVAL, "n_patches must be >= 1");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  const int64_t need = fvk::step_workspace_words(fvk::update_workgroups(dim, p, n));
  if (need > FV_NOALLOC_SCRATCH_WORDS)
    return fail(FV_EINVAL,
                "fv_step_gather_noalloc: %lld patches need %lld scratch words, the library "
                "holds %d; use fv_step_gather with a workspace",
                (long long)n, (long long)need, FV_NOALLOC_SCRATCH_WORDS);
  // every other argument is checked by the shared path before anything runs
  if (!patches || !neighbours || !q_in || !q_out || !dt_dev || !dt_next)
    return fail(FV_EINVAL, "null device pointer");
  unsigned long long* w = device_scratch((hipStream_t)stream);
  if (!w) return FV_EHIP;
  return step_gather_impl("fv_step_gather_noalloc", patches, n, neighbours, q_in, q_in_len,
                          q_out, q_out_len, dim, p, s, gamma, cfl, dt_dev, max_eig, dt_next,
                          lambda_out, reinterpret_cast<uint64_t*>(w),
                          (int64_t)FV_NOALLOC_SCRATCH_WORDS, stream);
}

int fv_step_gather_f32(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                       const float* q_in, int64_t q_in_len, float* q_out, int64_t q_out_len,
                       int dim, int p, int s, double gamma, double cfl, const double* dt_dev,
                       double* max_eig, double* dt_next, double* lambda_out,
                       uint64_t* workspace, int64_t workspace_words, void* stream) {
  return step_gather_impl("fv_step_gather_f32", patches, n, neighbours, q_in, q_in_len, q_out,
                          q_out_len, dim, p, s, gamma, cfl, dt_dev, max_eig, dt_next, lambda_out,
                          workspace, workspace_words, stream);
}

int fv_step_halo(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                 const double* q_in, int64_t q_in_len, double* q_out, int64_t q_out_len, int dim,
                 int p, int halo, int s, double gamma, double cfl, const double* dt_dev,
                 double* max_eig, double* dt_next, double* lambda_out, uint64_t* workspace,
                 int64_t workspace_words, void* stream) {
  int rc = check_shape(dim, p, halo, s);
  if (rc) return rc;
  if (n < 1) return fail(FV_EINVAL, "n_patches must be >= 1");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(FV_EINVAL, "cfl must be finite and > 0");
  if (!patches || !neighbours || !q_in || !q_out || !dt_dev || !dt_next || !workspace)
    return fail(FV_EINVAL, "null device pointer");
  if (dt_next == dt_dev) return fail(FV_EINVAL, "dt_next must not alias dt_dev");
  const int64_t need = fvk::step_workspace_words(fvk::update_workgroups(dim, p, n));
  if (workspace_words < need) return fail(FV_EINVAL, "workspace needs %lld words", (long long)need);
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  if ((rc = overlap_check(q_in, q_in_len, q_out, q_out_len))) return rc;
  fvk::CflOut co;
  co.cfl = cfl;
  co.dt_next = dt_next;
  co.lambda_out = lambda_out;
  co.ws = reinterpret_cast<unsigned long long*>(workspace);
  rc = fvk::launch_step_halo<double>(patches, n, neighbours, q_in, q_in_len, q_out, q_out_len,
                                     dim, p, gamma, dt_dev, max_eig, co, (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched("fv_step_halo");
}

int fv_max_eigenvalue(const fv_patch* patches, int64_t n, const double* q, int64_t q_len,
                      int q_halo, int which, int dim, int p, int s, double gamma,
                      double* per_patch, double* global, void* stream) {
  return max_eigenvalue_impl("fv_max_eigenvalue", patches, n, q, q_len, q_halo, which, dim, p, s,
                             gamma, per_patch, global, stream);
}

int fv_max_eigenvalue_f32(const fv_patch* patches, int64_t n, const float* q, int64_t q_len,
                          int q_halo, int which, int dim, int p, int s, double gamma,
                          double* per_patch, double* global, void* stream) {
  return max_eigenvalue_impl("fv_max_eigenvalue_f32", patches, n, q, q_len, q_halo, which, dim, p,
                             s, gamma, per_patch, global, stream);
}

int fv_conserved_totals(const fv_patch* patches, int64_t n, const double* q, int64_t q_len,
                        int q_halo, int which, int dim, int p, int s, double* per_patch,
                        double* totals, void* stream) {
  return totals_impl("fv_conserved_totals", patches, n, q, q_len, q_halo, which, dim, p, s,
                     per_patch, totals, stream);
}

int fv_conserved_totals_f32(const fv_patch* patches, int64_t n, const float* q, int64_t q_len,
                            int q_halo, int which, int dim, int p, int s, double* per_patch,
                            double* totals, void* stream) {
  return totals_impl("fv_conserved_totals_f32", patches, n, q, q_len, q_halo, which, dim, p, s,
                     per_patch, totals, stream);
}

int fv_cfl_timestep(const fv_patch* patches, int64_t n, const double* per_patch, int dim,
                    double cfl, double* lambda_out, double* dt_out, void* stream) {
  if (dim != 2 && dim != 3) return fail(FV_EINVAL, "dim must be 2 or 3");
  if (n < 1) return fail(FV_EINVAL, "n_patches must be >= 1");
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(FV_EINVAL, "cfl must be finite and > 0");
  if (!patches || !per_patch) return fail(FV_EINVAL, "null device pointer");
  if (!lambda_out && !dt_out) return ok();
  fvk::launch_reduce_cfl(patches, n, per_patch, dim, cfl, lambda_out, dt_out,
                         (hipStream_t)stream);
  return launched("fv_cfl_timestep");
}

int fv_fill_halo(const fv_patch* patches, int64_t n, const int64_t* neighbours, double* q,
                 int64_t q_len, int which, int dim, int p, int halo, int s, void* stream) {
  int rc = check_shape(dim, p, halo, s);
  if (rc) return rc;
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (which != FV_OFFSETS_IN && which != FV_OFFSETS_OUT)
    return fail(FV_EINVAL, "which_offsets must be FV_OFFSETS_IN or FV_OFFSETS_OUT");
  if (n == 0) return ok();
  if (!patches || !neighbours || !q) return fail(FV_EINVAL, "null device pointer");
  if (n * 2 * dim * (int64_t)(dim + 2) * ipow64(p, dim - 1) >= ((int64_t)1 << 39))
    return fail(FV_EINVAL, "batch too large for one halo launch");
  rc = fvk::launch_fill_halo_f64(patches, n, neighbours, q, q_len, which, dim, p,
                                 (hipStream_t)stream);
  if (rc) return fail(rc, "no kernel instance for dim=%d p=%d", dim, p);
  return launched("fv_fill_halo");
}

}  // extern "C"

namespace {

// ---- learned face-flux correction ------------------------------------------

int check_grid2(int npx, int npy, int p, int r, int bc) {
  if (npx < 1 || npy < 1 || p < 1) return fail(FV_EINVAL, "empty patch grid");
  if (r < 1 || p % r != 0) return fail(FV_EINVAL, "r must divide p (p=%d r=%d)", p, r);
  if (bc != 0 && bc != 1) return fail(FV_EINVAL, "bc must be 0 (periodic) or 1 (transmissive)");
  if ((int64_t)npx * npy * p * p > ((int64_t)1 << 31)) return fail(FV_EINVAL, "grid too large");
  return FV_OK;
}

}  // namespace

extern "C" {

int fv_learned_flux_accumulate(const double* q_fine, int npx, int npy, int p, int r, int bc,
                               double gamma, double weight, double* acc_x, double* acc_y,
                               void* stream) {
  int rc = check_grid2(npx, npy, p, r, bc);
  if (rc) return rc;
  if (!q_fine || !acc_x || !acc_y) return fail(FV_EINVAL, "null device pointer");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  fvk::launch_face_flux_accumulate(q_fine, npx, npy, p, r, bc, gamma, weight, acc_x, acc_y,
                                   (hipStream_t)stream);
  return launched("fv_learned_flux_accumulate");
}

int fv_learned_coarse_grain(const double* q_fine, int npx, int npy, int p, int r,
                            double* q_coarse, void* stream) {
  int rc = check_grid2(npx, npy, p, r, 0);
  if (rc) return rc;
  if (npx % r || npy % r) return fail(FV_EINVAL, "npx and npy must be multiples of r");
  if (!q_fine || !q_coarse) return fail(FV_EINVAL, "null device pointer");
  if (q_fine == q_coarse) return fail(FV_EINVAL, "q_coarse must not alias q_fine");
  fvk::launch_coarse_grain(q_fine, npx, npy, p, r, q_coarse, (hipStream_t)stream);
  return launched("fv_learned_coarse_grain");
}

int fv_learned_face_samples(const double* q_coarse, int npx, int npy, int p, int bc,
                            double gamma, const double* acc_x, const double* acc_y,
                            float* features, float* targets, float* indicator, void* stream) {
  int rc = check_grid2(npx, npy, p, 1, bc);
  if (rc) return rc;
  if (!q_coarse || !acc_x || !acc_y || !features || !targets || !indicator)
    return fail(FV_EINVAL, "null device pointer");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  fvk::launch_face_samples(q_coarse, npx, npy, p, bc, gamma, acc_x, acc_y, features, targets,
                           indicator, (hipStream_t)stream);
  return launched("fv_learned_face_samples");
}

int fv_mlp_fit_normalization(const float* x, int64_t x_rows, int cols, int mode,
                             const int64_t* rows, int64_t n_rows, float* mean_out,
                             float* scale_out, void* stream) {
  const int64_t n = rows ? n_rows : x_rows;
  if (x_rows < 1 || n < 1 || cols < 1 || cols > 65535) return fail(FV_EINVAL, "bad sizes");
  if (mode != 0 && mode != 1) return fail(FV_EINVAL, "mode must be 0 or 1");
  if (!x || !mean_out || !scale_out) return fail(FV_EINVAL, "null device pointer");
  fvk::launch_column_stats(x, x_rows, n, cols, mode, rows, mean_out, scale_out,
                           (hipStream_t)stream);
  return launched("fv_mlp_fit_normalization");
}

int fv_mlp_workspace_words(int batch) { return batch < 1 ? 0 : fvk::mlp_workspace_words(batch); }

int fv_mlp_train_step(float* blob, float* adam, int step, float lr, const float* features,
                      const float* targets, int64_t n_rows, const int64_t* batch_idx, int batch,
                      float* workspace, int64_t workspace_words, float* grad_out, void* stream) {
  if (n_rows < 1) return fail(FV_EINVAL, "n_rows must be >= 1");
  if (batch < 1 || batch > (1 << 20)) return fail(FV_EINVAL, "batch must be in [1, 2^20]");
  if (step < 1) return fail(FV_EINVAL, "step counts from 1");
  if (!(lr > 0.0f) || !isfinite(lr)) return fail(FV_EINVAL, "lr must be finite and > 0");
  if (!blob || !adam || !features || !targets || !batch_idx || !workspace)
    return fail(FV_EINVAL, "null device pointer");
  if (workspace_words < fvk::mlp_workspace_words(batch))
    return fail(FV_EINVAL, "workspace needs %d words", fvk::mlp_workspace_words(batch));
  fvk::launch_mlp_train_step(blob, adam, step, lr, features, targets, n_rows, batch_idx, batch,
                             workspace, grad_out, (hipStream_t)stream);
  return launched("fv_mlp_train_step");
}

int fv_mlp_forward(const float* blob, const float* features, int64_t n, float* out,
                   void* stream) {
  if (n < 0) return fail(FV_EINVAL, "n < 0");
  if (n == 0) return ok();
  if (!blob || !features || !out) return fail(FV_EINVAL, "null device pointer");
  if (n > ((int64_t)1 << 31)) return fail(FV_EINVAL, "too many samples");
  fvk::launch_mlp_forward(blob, features, n, out, (hipStream_t)stream);
  return launched("fv_mlp_forward");
}

int fv_batch_update_learned_2d(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                               const double* q_in, int64_t q_in_len, double* q_out,
                               int64_t q_out_len, double gamma, const double* dt_dev,
                               const float* blob, double threshold, double* max_eig,
                               void* stream) {
  if (n < 0) return fail(FV_EINVAL, "n_patches < 0");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(FV_EINVAL, "gamma must be > 1");
  if (!(threshold >= 0.0)) return fail(FV_EINVAL, "threshold must be >= 0");
  if (n == 0) return ok();
  if (!patches || !neighbours || !q_in || !q_out || !blob)
    return fail(FV_EINVAL, "null device pointer");
  if (q_in_len < 0 || q_out_len < 0) return fail(FV_EINVAL, "negative buffer length");
  if (n > (int64_t)0x7fffffff) return fail(FV_EINVAL, "too many patches for one launch");
  int rc = overlap_check(q_in, q_in_len, q_out, q_out_len);
  if (rc) return rc;
  fvk::launch_update_learned_2d(patches, n, neighbours, q_in, q_in_len, q_out, q_out_len, gamma,
                                dt_dev, blob, threshold, max_eig, (hipStream_t)stream);
  return launched("fv_batch_update_learned_2d");
}

}  // extern "C"
