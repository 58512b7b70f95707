// The no-allocation entry point: lco_permute for callers that cannot allocate
// device memory.  Its temporary memory is a fixed workspace inside the library,
// one per device, that lives until the process ends.
#include <mutex>

#include "lco_internal.h"

namespace lco {
lco_status set_error(const Error& e);
lco_status set_error_msg(lco_status s, const char* msg);
}  // namespace lco

using namespace lco;

namespace {

// The workspace.  In host code this name is not a device address: host code
// uses only the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[LCO_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // scratch's address on each device (set once per device)

void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return device >= 0 && device < kMaxDevices ? g_ptr[device] : nullptr;
}

}  // namespace

namespace lco {

void noalloc_init_device(int device) {
  if (device < 0 || device >= kMaxDevices) fail(LCO_E_ARG, "no-allocation workspace: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  hip_check(e, "hipGetSymbolAddress(scratch)");
  if (!ptr) fail(LCO_E_HIP, "no-allocation workspace: the device has no address for it");
  g_ptr[device] = ptr;
}

}  // namespace lco

extern "C" lco_status lco_permute_noalloc(lco_ctx ctx, lco_tensor in, const int* perm, uint64_t* out_livs,
                                          double* out_vals, uint64_t* out_dims) {
  try {
    if (!ctx || !in || !perm || !out_dims) fail(LCO_E_ARG, "lco_permute_noalloc: NULL argument");
    if (in->ctx->device != ctx->device) fail(LCO_E_ARG, "lco_permute_noalloc: tensor lives on another device");
    if (in->nnz > LCO_NOALLOC_MAX_NNZ)
      fail(LCO_E_UNSUPPORTED, "lco_permute_noalloc: more than LCO_NOALLOC_MAX_NNZ (2^20) non-zeros");
    if (in->nnz > 0 && (!out_livs || !out_vals)) fail(LCO_E_ARG, "lco_permute_noalloc: output array is NULL");
    const RpDetail plan = plan_permute(in->order, in->dims, perm, in->nnz, default_digit_cap());
    void* ws = scratch_of(ctx->device);
    if (!ws) fail(LCO_E_HIP, "lco_permute_noalloc: no workspace on this device (context not created)");
    LCO_HIP(hipSetDevice(ctx->device));
    {
      FixedScratch fixed(ctx, ws, LCO_NOALLOC_SCRATCH_BYTES);
      permute_storage(ctx, in, plan, out_livs, out_vals);
    }
    for (int r = 0; r < in->order; ++r) out_dims[r] = plan.new_dims[r];
    return LCO_OK;
  } catch (const Error& e) {
    return set_error(e);
  } catch (const std::exception& e) {
    return set_error_msg(LCO_E_HIP, e.what());
  }
}
