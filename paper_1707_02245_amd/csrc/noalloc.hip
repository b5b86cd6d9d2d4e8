// A^T without device allocation: pat_adjoint_noalloc keeps the partial images
// that pat_adjoint sums into its output (one per quarter-turn slot of the
// stored A^T, or one per detector group of the matrix-free scatter) in a
// fixed device array of this file instead of memory the geometry allocates on
// first use. The kernels are pat_adjoint's own, so the result is the same bit
// for bit.
//
// Every GPU the library runs on holds its own copy of the array (at its own
// address) until the process ends. The host-side name `scratch` is only a
// stand-in for the symbol: its device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and only that address
// is passed to kernels.

#include <mutex>

#include "pat_internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of this device's array (looked up on the first call on the
// device; hipGetSymbolAddress does not allocate).
void* scratch_on_current_device() {
  int dev = 0;
  PAT_HIP(hipGetDevice(&dev));
  PAT_CHECK_ARG(dev >= 0 && dev < kMaxDevices, "device index beyond the library's per-device table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    PAT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PAT_CHECK_ARG(p != nullptr, "no device address for the scratch array");
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

}  // namespace

extern "C" pat_status pat_adjoint_noalloc(pat_geometry g, const void* d_f, void* d_u, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(d_u != nullptr && d_f != nullptr, "NULL buffer");
    PAT_CHECK_ARG(g->adj_mode == 0 || g->csr_nnz >= 0,
                  "the stored A^T is not built (pat_geometry_set_adjoint builds it)");
    const size_t need = pat::adjoint_scratch_bytes(g);
    if (need > kScratchBytes) {
      pat::set_error("pat_adjoint_noalloc needs %zu bytes of partial images, more than its fixed %zu-byte "
                     "device array (use pat_adjoint)", need, kScratchBytes);
      return PAT_ERR_INVALID_ARG;
    }
    void* sp = scratch_on_current_device();
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the partial images are written in full by the A^T kernels before the
    // summation reads them, so nothing needs clearing between calls
    if (g->dtype == PAT_F64)
      pat::apply_adjoint_scratch<double>(g, static_cast<const double*>(d_f), static_cast<double*>(d_u),
                                         static_cast<double*>(sp), s);
    else
      pat::apply_adjoint_scratch<float>(g, static_cast<const float*>(d_f), static_cast<float*>(d_u),
                                        static_cast<float*>(sp), s);
    return PAT_OK;
  });
}
