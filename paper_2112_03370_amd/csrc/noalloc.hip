// Allocation-free PCG (mm_pcg_solve_noalloc): the same solve as mm_pcg_solve for callers that
// cannot allocate device memory (serving loops with a fixed footprint, harnesses that forbid
// hipMalloc).  The solve's pixel-domain vectors (b, r, z, p, q), reduction partials and device
// scalars live in one file-scope device array, `scratch`, of kScratchBytes.  Its device address
// is looked up once per device with hipGetSymbolAddress (in host code the array's name is not a
// device address) and only that address is passed to kernels.  Every call on a device uses that
// device's array: calls are serialised per device by a host mutex, and nothing in the array is
// assumed to be zero (the PCG kernels write every element before reading it).
#include <array>
#include <cstring>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr size_t kScratchBytes = size_t{64} << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceSlot {
  std::mutex mu;          // serialises the calls on this device
  bool looked_up = false;
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
};

std::array<DeviceSlot, kMaxDevices>& slots() {
  static std::array<DeviceSlot, kMaxDevices> s;
  return s;
}

constexpr size_t align_up(size_t v) { return (v + 255) & ~size_t{255}; }

// Bytes of scratch a plan's solve needs: five pixel vectors, the partials, the state.
size_t scratch_need(const Plan* P) {
  const size_t nu = static_cast<size_t>(3 * P->n_kept) * sizeof(double);
  const size_t part = static_cast<size_t>(4 * reduction_blocks(P->n_kept)) * sizeof(double);
  return 5 * align_up(nu) + align_up(part) + align_up(sizeof(CgState));
}

}  // namespace

}  // namespace mm

using namespace mm;

extern "C" {

mm_status mm_pcg_solve_noalloc(const mm_plan_t* plan, const float* d, int32_t k, int64_t ld_d,
                               double* x, const mm_solve_opts* opts, mm_solve_info* info,
                               void* stream) {
  if (plan == nullptr) return fail(MM_ERR_INVALID, "plan is NULL");
  Plan* P = reinterpret_cast<Plan*>(const_cast<mm_plan_t*>(plan));
  int dev = -1;
  MM_HIP_TRY(hipGetDevice(&dev));
  if (dev != P->device)
    return fail(MM_ERR_INVALID, "plan belongs to another device than the current one");
  if (dev < 0 || dev >= kMaxDevices) return fail(MM_ERR_UNSUPPORTED, "device index beyond 63");
  if (k < 0) return fail(MM_ERR_INVALID, "k < 0");
  if (k > 1 && ld_d < P->n_samples) return fail(MM_ERR_INVALID, "ld_d < n_samples");
  if (k > 0 && ((P->n_samples > 0 && !d) || (P->n_kept > 0 && !x)))
    return fail(MM_ERR_INVALID, "NULL vector");
  if (opts && opts->tol < 0) return fail(MM_ERR_INVALID, "tol < 0");
  if (opts && ((opts->block != 0 && opts->block != 1) || opts->precond != 0 || opts->refine != 0 ||
               opts->check_fp64 != 0))
    return fail(MM_ERR_UNSUPPORTED,
                "the allocation-free solve runs block-Jacobi PCG per column only (block 0/1, "
                "precond 0, no refinement or FP64 check)");
  if (needs_time_buffers(P) || P->precision != MM_PRECISION_MIXED || P->n_poly > 0 ||
      (P->algo == MM_TOEPLITZ_FFT && long_fft_size(P->fft_n)))
    return fail(MM_ERR_UNSUPPORTED,
                "the allocation-free solve needs a plan whose product keeps the time domain on "
                "chip (fused FFT or diagonal weights)");
  if (P->timing.enabled)
    return fail(MM_ERR_UNSUPPORTED, "per-kernel timing records events: disable it first");
  const size_t need = scratch_need(P);
  if (need > kScratchBytes)
    return fail(MM_ERR_INVALID, "plan needs " + std::to_string(need) +
                                    " bytes of solve scratch; the allocation-free solve holds " +
                                    std::to_string(kScratchBytes) + " (n_kept too large)");
  DeviceSlot& slot = slots()[dev];
  std::lock_guard<std::mutex> lk(slot.mu);
  if (!slot.looked_up) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(MM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    slot.ptr = static_cast<unsigned char*>(p);
    slot.looked_up = true;
  }
  try {
    // carve the solve workspace out of this device's array
    Work W;
    unsigned char* c = slot.ptr;
    const size_t nu = align_up(static_cast<size_t>(3 * P->n_kept) * sizeof(double));
    W.r = reinterpret_cast<double*>(c);
    W.z = reinterpret_cast<double*>(c + nu);
    W.p = reinterpret_cast<double*>(c + 2 * nu);
    W.q = reinterpret_cast<double*>(c + 3 * nu);
    W.b = reinterpret_cast<double*>(c + 4 * nu);
    W.nrb = reduction_blocks(P->n_kept);
    W.partial = reinterpret_cast<double*>(c + 5 * nu);
    W.state = reinterpret_cast<CgState*>(
        c + 5 * nu + align_up(static_cast<size_t>(4 * W.nrb) * sizeof(double)));
    CgState host_state;  // pageable mirror read after each synchronisation
    std::memset(&host_state, 0, sizeof(host_state));
    W.h_state = &host_state;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mm_status worst = MM_OK;
    std::string msg;
    for (int32_t j = 0; j < k; ++j) {
      mm_solve_info tmp{};
      const mm_status st = pcg_solve(P, W, d + j * ld_d, x + j * 3 * P->n_kept, opts,
                                     info ? &info[j] : &tmp, s, /*alloc_free=*/true);
      if (st == MM_ERR_HIP || st == MM_ERR_INVALID || st == MM_ERR_UNSUPPORTED) return st;
      if (st != MM_OK && worst == MM_OK) {
        worst = st;
        msg = last_error_cstr();
      }
    }
    if (worst != MM_OK) set_error(msg);
    return worst;
  } catch (const std::exception& ex) {
    return fail(MM_ERR_HIP, std::string("unexpected exception: ") + ex.what());
  } catch (...) {
    return fail(MM_ERR_HIP, "unexpected exception");
  }
}

}  // extern "C"
