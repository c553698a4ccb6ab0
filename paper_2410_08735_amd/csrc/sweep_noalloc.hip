// rte_sweep_noalloc: the batched transport sweep and its quadrature reduction
// (section 3.1) with the partial scalar fluxes in a file-scope device array
// instead of library-allocated memory, for callers that cannot allocate.
#include <mutex>

#include "rte_internal.h"

namespace rte {

// 64 MiB of partial scalar fluxes, one copy per GPU for the life of the
// process.  Host code never passes this name to a kernel: it is a host-side
// stand-in, and only the address hipGetSymbolAddress returns for a device is
// valid there.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device, looked up once per
// device (with that device current).
static int scratch_ptr(void** out) {
  int dev = 0;
  RTE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return RTE_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      std::fprintf(stderr, "rte_sweep_noalloc: hipGetSymbolAddress failed on device %d: %s\n", dev,
                   hipGetErrorString(e));
      return RTE_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RTE_OK;
}

}  // namespace rte

extern "C" int rte_sweep_noalloc(const rte_batch* cb, const double* sigma_t, const double* q,
                                 const double* inflow, double* phi_out, int dtype, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  const int prec = dtype == RTE_F32 ? 1 : (dtype == RTE_F64 ? 0 : -1);
  if (!b || !sigma_t || !q || !phi_out || prec < 0) return RTE_EINVAL;
  const rte::Plan& p = b->plan[prec];
  const size_t need = (size_t)p.part_elems * (prec == 0 ? sizeof(double) : sizeof(float));
  if (need > rte::NOALLOC_SCRATCH_BYTES) {
    std::fprintf(stderr,
                 "rte_sweep_noalloc: this batch's sweep plan needs %zu bytes of partial fluxes, above the "
                 "%zu-byte static scratch limit (use rte_sweep)\n",
                 need, rte::NOALLOC_SCRATCH_BYTES);
    return RTE_EINVAL;
  }
  void* part = nullptr;
  RTE_TRY(rte::scratch_ptr(&part));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // no autotuning (it allocates) and no profiler events: the current plan as is
  RTE_TRY(rte::sweep_launch(b, prec, sigma_t, nullptr, nullptr, q, inflow, nullptr, s, nullptr, -2.0, part));
  return rte::reduce_partials(b, prec, 1.0, nullptr, 0.0, phi_out, s, nullptr, nullptr, 0.0, part);
}
