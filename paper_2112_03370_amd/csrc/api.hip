// C ABI entry points: argument validation, dispatch, error reporting, per-kernel timing.
#include <cstring>
#include <exception>
#include <new>

#include "mm_internal.h"

namespace mm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

const char* last_error_cstr() { return g_last_error.c_str(); }

mm_status fail(mm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

TimedLaunch::TimedLaunch(Plan* plan, int k, hipStream_t st) : P(plan), kind(k), s(st) {
  if (!P->timing.enabled) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}

TimedLaunch::~TimedLaunch() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  P->timing.pending[kind].push_back(TimedPair{e0, e1, P->timing.tag});
}

void timing_drop_range(Plan* P, int32_t first, int32_t last) {
  for (int k = 0; k < K_NKINDS; ++k) {
    auto& v = P->timing.pending[k];
    std::vector<TimedPair> keep;
    for (const TimedPair& t : v) {
      if (t.tag >= first && t.tag <= last) {
        (void)hipEventSynchronize(t.e1);
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
      } else {
        keep.push_back(t);
      }
    }
    v.swap(keep);
  }
}

}  // namespace mm

using namespace mm;

namespace {

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline Plan* as_plan(const mm_plan_t* p) {
  return reinterpret_cast<Plan*>(const_cast<mm_plan_t*>(p));
}

mm_status check_plan(const mm_plan_t* p) {
  if (p == nullptr) return fail(MM_ERR_INVALID, "plan is NULL");
  return MM_OK;
}

mm_status check_device(const Plan* P) {
  int dev = -1;
  MM_HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device)
    return fail(MM_ERR_INVALID, "plan belongs to device " + std::to_string(P->device) +
                                    " but the current device is " + std::to_string(dev));
  return MM_OK;
}

template <class F>
mm_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(MM_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(MM_ERR_HIP, std::string("unexpected exception: ") + e.what());
  } catch (...) {
    return fail(MM_ERR_HIP, "unexpected exception");
  }
}

mm_status drain_timing(Plan* P) {
  for (int k = 0; k < K_NKINDS; ++k) {
    auto& v = P->timing.pending[k];
    for (const TimedPair& t : v) {
      MM_HIP_TRY(hipEventSynchronize(t.e1));
      float ms = 0.0f;
      MM_HIP_TRY(hipEventElapsedTime(&ms, t.e0, t.e1));
      P->timing.total_ms[k] += ms;
      P->timing.count[k] += 1;
      (void)hipEventDestroy(t.e0);
      (void)hipEventDestroy(t.e1);
    }
    v.clear();
  }
  return MM_OK;
}

}  // namespace

extern "C" {

mm_status mm_plan(const mm_geometry* g, void* stream, mm_plan_t** out) {
  if (out == nullptr) return fail(MM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (g == nullptr) return fail(MM_ERR_INVALID, "geometry is NULL");
  return guarded([&]() -> mm_status {
    Plan* P = nullptr;
    MM_TRY(build_plan(g, as_stream(stream), &P));
    *out = reinterpret_cast<mm_plan_t*>(P);
    return MM_OK;
  });
}

mm_status mm_plan_destroy(mm_plan_t* plan) {
  if (plan == nullptr) return MM_OK;
  destroy_plan(as_plan(plan));
  return MM_OK;
}

mm_status mm_plan_info(const mm_plan_t* plan, mm_plan_info_t* out) {
  MM_TRY(check_plan(plan));
  if (out == nullptr) return fail(MM_ERR_INVALID, "out is NULL");
  const Plan* P = as_plan(plan);
  std::memset(out, 0, sizeof(*out));
  out->n_samples = P->n_samples;
  out->n_pix_global = P->n_pix_global;
  out->n_obs = P->n_obs;
  out->n_kept = P->n_kept;
  out->n_excised = P->n_obs - P->n_kept;
  out->n_gap_samples = P->n_gap;
  out->device_bytes = P->device_bytes;
  out->lambda_max = P->lambda_max;
  out->toeplitz_algo = P->algo;
  out->fft_size = P->algo == MM_TOEPLITZ_FFT ? P->fft_n : 0;
  out->n_blocks = P->n_blocks;
  out->n_chunks = P->n_chunks;
  out->fused = (P->lambda_max > 0 && P->algo == MM_TOEPLITZ_FFT && P->fused)
                   ? (long_fft_size(P->fft_n) ? 3 : (P->reg_fft ? 2 : 1))
                   : 0;
  out->precision = P->precision;
  out->n_poly = P->n_poly;
  out->n_baselines = P->n_baselines;
  return MM_OK;
}

mm_status mm_plan_pixels(const mm_plan_t* plan, int64_t* global_ids, int32_t* hits) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (P->n_kept == 0) return MM_OK;
  if (global_ids)
    MM_HIP_TRY(hipMemcpy(global_ids, P->kept_ids, P->n_kept * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (hits) MM_HIP_TRY(hipMemcpy(hits, P->hits, P->n_kept * sizeof(int32_t), hipMemcpyDeviceToHost));
  return MM_OK;
}

mm_status mm_unpoint(const mm_plan_t* plan, const double* x, float* t, void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if ((P->n_kept > 0 && !x) || (P->n_samples > 0 && !t)) return fail(MM_ERR_INVALID, "NULL vector");
  return guarded([&]() -> mm_status { return launch_unpoint(P, x, t, nullptr, as_stream(stream)); });
}

mm_status mm_noise_weight(const mm_plan_t* plan, const float* t, float* u, void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (P->n_samples > 0 && (!t || !u)) return fail(MM_ERR_INVALID, "NULL vector");
  if (P->n_samples > 0 && t == u) return fail(MM_ERR_INVALID, "t and u must not alias");
  return guarded([&]() -> mm_status { return launch_noise_weight(P, t, u, P->work.scratch, nullptr, as_stream(stream)); });
}

mm_status mm_point(const mm_plan_t* plan, const float* u, double* y, void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if ((P->n_kept > 0 && !y) || (P->n_samples > 0 && !u)) return fail(MM_ERR_INVALID, "NULL vector");
  return guarded([&]() -> mm_status { return launch_point(P, u, y, true, nullptr, as_stream(stream)); });
}

mm_status mm_rhs(const mm_plan_t* plan, const float* d, int32_t k, int64_t ld_d, double* b,
                 void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (k < 0) return fail(MM_ERR_INVALID, "k < 0");
  if (k > 1 && ld_d < P->n_samples) return fail(MM_ERR_INVALID, "ld_d < n_samples");
  if (k > 0 && ((P->n_samples > 0 && !d) || (P->n_kept > 0 && !b))) return fail(MM_ERR_INVALID, "NULL vector");
  hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lock(P->mu);
  return guarded([&]() -> mm_status {
    for (int32_t j = 0; j < k; ++j) MM_TRY(compute_rhs(P, P->work, d + j * ld_d, b + j * 3 * P->n_kept, s));
    return MM_OK;
  });
}

mm_status mm_apply_A(const mm_plan_t* plan, const double* x, double* y, int32_t k, void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (k < 0) return fail(MM_ERR_INVALID, "k < 0");
  if (k > 0 && P->n_kept > 0 && (!x || !y)) return fail(MM_ERR_INVALID, "NULL vector");
  if (k > 0 && P->n_kept > 0 && x == y) return fail(MM_ERR_INVALID, "x and y must not alias");
  hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lock(P->mu);
  return guarded([&]() -> mm_status {
    return apply_A_multi(P, P->work, x, 3 * P->n_kept, y, 3 * P->n_kept, k, s);
  });
}

mm_status mm_precond_bj(const mm_plan_t* plan, const double* r, double* z, int32_t k,
                        void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (k < 0) return fail(MM_ERR_INVALID, "k < 0");
  if (k > 0 && P->n_kept > 0 && (!r || !z)) return fail(MM_ERR_INVALID, "NULL vector");
  hipStream_t s = as_stream(stream);
  return guarded([&]() -> mm_status {
    for (int32_t j = 0; j < k; ++j)
      MM_TRY(launch_precond(P, r + j * 3 * P->n_kept, z + j * 3 * P->n_kept, s));
    return MM_OK;
  });
}

mm_status mm_pcg_solve(const mm_plan_t* plan, const float* d, int32_t k, int64_t ld_d, double* x,
                       const mm_solve_opts* opts, mm_solve_info* info, void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (k < 0) return fail(MM_ERR_INVALID, "k < 0");
  if (k > 1 && ld_d < P->n_samples) return fail(MM_ERR_INVALID, "ld_d < n_samples");
  if (k > 0 && ((P->n_samples > 0 && !d) || (P->n_kept > 0 && !x))) return fail(MM_ERR_INVALID, "NULL vector");
  if (opts && opts->tol < 0) return fail(MM_ERR_INVALID, "tol < 0");
  if (opts && opts->refine < 0) return fail(MM_ERR_INVALID, "refine < 0");
  hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lock(P->mu);
  return guarded([&]() -> mm_status {
    if (opts && opts->precond != 0 && opts->precond != 1) return fail(MM_ERR_INVALID, "precond must be 0 or 1");
    if (opts && (opts->refine > 0 || opts->check_fp64) && opts->block != 0 && opts->block != 1 && k > 1)
      return fail(MM_ERR_UNSUPPORTED, "refine and check_fp64 apply to block 0/1 solves");
    if (opts && opts->precond == 1 && P->defl.m == 0)
      return fail(MM_ERR_INVALID, "precond = 1 needs mm_deflation_build first");
    if (opts && opts->block != 0 && opts->block != 1 && k > 0) {
      if (opts->use_x0) return fail(MM_ERR_INVALID, "use_x0 is not supported with block != 0/1");
      if (opts->precond == 1) return fail(MM_ERR_UNSUPPORTED, "stacked solves use block-Jacobi");
      return block_solve(P, P->work, d, k, ld_d, x, opts, info, s);
    }
    mm_status worst = MM_OK;
    std::string msg;
    for (int32_t j = 0; j < k; ++j) {
      mm_solve_info tmp{};
      mm_status st = pcg_solve(P, P->work, d + j * ld_d, x + j * 3 * P->n_kept, opts, info ? &info[j] : &tmp, s);
      if (st == MM_ERR_HIP || st == MM_ERR_OOM || st == MM_ERR_INVALID || st == MM_ERR_UNSUPPORTED)
        return st;
      if (st != MM_OK && worst == MM_OK) {
        worst = st;
        msg = mm_last_error();
      }
    }
    if (worst != MM_OK) set_error(msg);
    return worst;
  });
}

mm_status mm_deflation_build(mm_plan_t* plan, const float* d, int32_t m, void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (m < 1 || m > kMaxDeflation) return fail(MM_ERR_INVALID, "m out of [1, 128]");
  if (P->n_samples > 0 && !d) return fail(MM_ERR_INVALID, "NULL data");
  if (P->n_kept == 0) return fail(MM_ERR_INVALID, "plan has no kept pixels");
  std::lock_guard<std::mutex> lock(P->mu);
  return guarded([&]() -> mm_status { return deflation_build(P, d, m, as_stream(stream)); });
}

mm_status mm_deflation_info(const mm_plan_t* plan, mm_deflation_info_t* out) {
  MM_TRY(check_plan(plan));
  if (!out) return fail(MM_ERR_INVALID, "out is NULL");
  const Plan* P = as_plan(plan);
  out->m = P->defl.m;
  out->rank = P->defl.rank;
  out->e_min = P->defl.e_min;
  out->e_max = P->defl.e_max;
  out->build_ms = P->defl.build_ms;
  out->device_bytes = P->defl.bytes;
  return MM_OK;
}

mm_status mm_deflation_clear(mm_plan_t* plan) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  std::lock_guard<std::mutex> lock(P->mu);
  deflation_free(&P->defl);
  return MM_OK;
}

mm_status mm_deflation_vectors(const mm_plan_t* plan, double* z, void* stream) {
  MM_TRY(check_plan(plan));
  const Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (P->defl.m == 0) return fail(MM_ERR_INVALID, "no deflation space built");
  if (!z) return fail(MM_ERR_INVALID, "NULL output");
  const size_t bytes = sizeof(double) * static_cast<size_t>(P->defl.m) * 3 * P->n_kept;
  return guarded([&]() -> mm_status {
    MM_HIP_TRY(hipMemcpyAsync(z, P->defl.Z, bytes, hipMemcpyDeviceToDevice, as_stream(stream)));
    return MM_OK;
  });
}

mm_status mm_precond_2lvl(const mm_plan_t* plan, const double* r, double* z, int32_t k,
                          void* stream) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(check_device(P));
  if (k < 0) return fail(MM_ERR_INVALID, "k < 0");
  if (P->defl.m == 0) return fail(MM_ERR_INVALID, "no deflation space built");
  if (k > 0 && (!r || !z)) return fail(MM_ERR_INVALID, "NULL vector");
  if (k > 0 && r == z) return fail(MM_ERR_INVALID, "r and z must not alias");
  hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lock(P->mu);
  return guarded([&]() -> mm_status {
    const int64_t nu = 3 * P->n_kept;
    for (int32_t j = 0; j < k; ++j)
      MM_TRY(deflation_apply(P, r + j * nu, z + j * nu, nullptr, P->work.partial, P->work.nrb,
                             nullptr, s));
    return MM_OK;
  });
}

mm_status mm_set_timing(mm_plan_t* plan, int32_t enable) {
  MM_TRY(check_plan(plan));
  Plan* P = as_plan(plan);
  MM_TRY(drain_timing(P));
  P->timing.enabled = enable != 0;
  for (int k = 0; k < K_NKINDS; ++k) {
    P->timing.total_ms[k] = 0.0;
    P->timing.count[k] = 0;
  }
  return MM_OK;
}

mm_status mm_kernel_time(mm_plan_t* plan, int32_t kind, double* total_ms, int64_t* launches) {
  MM_TRY(check_plan(plan));
  if (kind < 0 || kind >= K_NKINDS) return fail(MM_ERR_INVALID, "unknown kernel kind");
  Plan* P = as_plan(plan);
  MM_TRY(drain_timing(P));
  if (total_ms) *total_ms = P->timing.total_ms[kind];
  if (launches) *launches = P->timing.count[kind];
  return MM_OK;
}

const char* mm_status_string(mm_status s) {
  switch (s) {
    case MM_OK: return "MM_OK";
    case MM_PENDING: return "MM_PENDING";
    case MM_ERR_INVALID: return "MM_ERR_INVALID";
    case MM_ERR_NOT_SPD: return "MM_ERR_NOT_SPD";
    case MM_ERR_NO_CONV: return "MM_ERR_NO_CONV";
    case MM_ERR_OOM: return "MM_ERR_OOM";
    case MM_ERR_HIP: return "MM_ERR_HIP";
    case MM_ERR_BUDGET: return "MM_ERR_BUDGET";
    case MM_ERR_UNSUPPORTED: return "MM_ERR_UNSUPPORTED";
    case MM_ERR_NOT_FOUND: return "MM_ERR_NOT_FOUND";
    default: return "MM_UNKNOWN_STATUS";
  }
}

const char* mm_last_error(void) { return mm::last_error_cstr(); }

}  // extern "C"
