// C-ABI entry points for the transport operators (sections 2.3, 3.1, 3.2).
#include "rte_internal.h"


static inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

static int prec_of(int dtype) { return dtype == RTE_F32 ? 1 : (dtype == RTE_F64 ? 0 : -1); }

extern "C" int rte_sweep(const rte_batch* cb, const double* sigma_t, const double* q,
                         const double* inflow, double* phi_out, double* psi_out, int dtype,
                         void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  const int prec = prec_of(dtype);
  if (!b || !sigma_t || !q || (!phi_out && !psi_out) || prec < 0) return RTE_EINVAL;
  hipStream_t s = as_stream(stream);
  RTE_TRY(rte::autotune_sweep(b, prec, sigma_t, s));
  RTE_TRY(rte::sweep_launch(b, prec, sigma_t, nullptr, nullptr, q, inflow, psi_out, s));
  if (phi_out) RTE_TRY(rte::reduce_partials(b, prec, 1.0, nullptr, 0.0, phi_out, s));
  return RTE_OK;
}

extern "C" int rte_scalar_flux(const rte_batch* cb, const double* psi, double* phi_out,
                               void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !psi || !phi_out) return RTE_EINVAL;
  return rte::scalar_flux(b, psi, phi_out, as_stream(stream));
}

extern "C" int rte_apply_A(const rte_batch* cb, const double* sigma_t, const double* sigma_s,
                           const double* x, double* y, int dtype, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  const int prec = prec_of(dtype);
  if (!b || !sigma_t || !sigma_s || !x || !y || prec < 0) return RTE_EINVAL;
  hipStream_t s = as_stream(stream);
  RTE_TRY(rte::autotune_sweep(b, prec, sigma_t, s));
  RTE_TRY(rte::sweep_launch(b, prec, sigma_t, sigma_s, x, nullptr, nullptr, nullptr, s));
  return rte::reduce_partials(b, prec, -1.0, x, 1.0, y, s);
}

extern "C" int rte_rhs(const rte_batch* cb, const double* sigma_t, const double* G,
                       const double* inflow, double* b_out, int dtype, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  const int prec = prec_of(dtype);
  if (!b || !sigma_t || !G || !b_out || prec < 0) return RTE_EINVAL;
  hipStream_t s = as_stream(stream);
  RTE_TRY(rte::autotune_sweep(b, prec, sigma_t, s));
  RTE_TRY(rte::sweep_launch(b, prec, sigma_t, nullptr, nullptr, G, inflow, nullptr, s));
  return rte::reduce_partials(b, prec, 1.0, nullptr, 0.0, b_out, s);
}

extern "C" int rte_batch_set_sweep_plan(rte_batch* b, int dtype, int variant, int G, int opl, int threads) {
  return rte::set_sweep_plan(b, prec_of(dtype), variant, G, opl, threads);
}

extern "C" int rte_batch_sweep_plan(const rte_batch* b, int dtype, int32_t* out) {
  const int prec = prec_of(dtype);
  if (!b || prec < 0 || !out) return RTE_EINVAL;
  const rte::Plan& p = b->plan[prec];
  out[0] = p.variant;
  out[1] = p.G;
  out[2] = p.opl;
  out[3] = p.threads;
  out[4] = p.tuned ? 1 : 0;
  out[5] = p.order;
  return RTE_OK;
}

extern "C" int rte_batch_set_sweep_order(rte_batch* b, int dtype, int order) {
  return rte::set_sweep_order(b, prec_of(dtype), order);
}
