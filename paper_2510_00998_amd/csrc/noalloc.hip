// hpmg_smooth_noalloc: block-Jacobi smoothing (projection + fused sweeps, as
// hpmg_smooth) with its two ping-pong trace buffers in a file-scope device
// array instead of memory the library allocates, for callers that cannot
// allocate device memory during the call (code under stream capture, serving
// loops, harnesses that forbid it).
//
// The array exists once per GPU for the lifetime of the process.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the device symbol): hpmg_setup resolves the device address
// once per device with hipGetSymbolAddress while that device is current, and
// every use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hpmg.h"
#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = HPMG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t round_up_256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

namespace hpmg {
namespace detail {

// Device address of this device's scratch array, resolved on the first call
// per device (with that device current).
void init_noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) throw HpmgError(HPMG_E_DEVICE, "device ordinal beyond 63");
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw HpmgError(HPMG_E_DEVICE, "hipGetSymbolAddress returned a null address for the scratch array");
  g_scratch_ptr[dev] = p;
}

}  // namespace detail
}  // namespace hpmg

using namespace hpmg::detail;

extern "C" hpmg_status hpmg_smooth_noalloc(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nsweeps,
                                           int nrhs, hipStream_t stream) {
  try {
    require(h && u && b, "NULL argument");
    require(nrhs >= 1 && nrhs <= h->opt.max_rhs, "nrhs out of range");
    require(nsweeps >= 0, "nsweeps must be >= 0");
    require(dtype >= HPMG_F64 && dtype <= HPMG_BF16, "bad dtype");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    require(dev == h->dev, "the handle's device is not the current device");
    void* base = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      base = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
    }
    if (!base) throw HpmgError(HPMG_E_DEVICE, "scratch array not resolved on this device");
    if (nsweeps == 0) return HPMG_OK;
    h->trace_state[dtype] = -1;  // u changes; the handle's own traces no longer describe it
    DGLevel& L = h->dg[0];
    const size_t esz = dtype == HPMG_F64 ? 8 : (dtype == HPMG_F32 ? 4 : 2);
    const size_t per = round_up_256(L.trsize * (size_t)nrhs * esz);
    if (2 * per > kScratchBytes)
      throw HpmgError(HPMG_E_INVALID, "hpmg_smooth_noalloc: the two trace buffers need " + std::to_string(2 * per) +
                                          " bytes, more than the " + std::to_string(kScratchBytes) +
                                          "-byte static scratch array (use hpmg_smooth)");
    auto run = [&](auto tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      T* tr[2] = {(T*)base, (T*)((unsigned char*)base + per)};
      hpmg::DGArgs<T> pa = dg_args<T>(h, L);
      pa.u_in = (const T*)u;
      pa.tr_out = tr[0];
      dg_run(h, hpmg::OP_PROJECT, pa, L.N, nrhs, 0, stream);
      for (int k = 0; k < nsweeps; ++k) {
        hpmg::DGArgs<T> a = dg_args<T>(h, L);
        a.u_in = (T*)u;
        a.u_out = (T*)u;
        a.b = (const T*)b;
        a.tr_in = tr[k & 1];
        a.tr_out = tr[(k + 1) & 1];
        dg_run(h, hpmg::OP_SWEEP, a, L.N, nrhs, 0, stream);
      }
    };
    switch (dtype) {
      case HPMG_F64: run((double*)nullptr); break;
      case HPMG_F32: run((float*)nullptr); break;
      case HPMG_F16: run((_Float16*)nullptr); break;
      default: run((__bf16*)nullptr); break;
    }
    return HPMG_OK;
  } catch (const HpmgError& e) {
    set_last_error(e.what());
    return e.st;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HPMG_E_INVALID;
  }
}
