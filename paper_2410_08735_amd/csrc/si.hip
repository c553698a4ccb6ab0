// Source iteration with synthetic acceleration (section 3): the left-
// preconditioned Richardson iteration on the memory-efficient system,
//   r^(l) = phi^(l,*) - phi^(l-1) = b~ - A~ phi^(l-1)   (one batched sweep),
//   phi^(l) = phi^(l-1) + M_l^{-1} r^(l),
// with M_l the ROMSAD switch (M_ROM for l <= window, M_DSA after it), DSA
// alone, or no acceleration.  Stops per instance when ||r|| <= rtol ||b~||.
#include <algorithm>
#include <vector>

#include "fgmres.h"

namespace rte {

struct SiWork {
  rte_batch* b = nullptr;
  Space sp;
  double *btil = nullptr, *r = nullptr, *z = nullptr, *norms = nullptr, *part = nullptr;
  int32_t* act = nullptr;
  int init(rte_batch* batch) {
    b = batch;
    std::vector<int64_t> lens(b->n_inst);
    for (int k = 0; k < b->n_inst; ++k) lens[k] = rte_batch_ndof(b, k);
    RTE_TRY(sp.init(lens));
    const int64_t tot = b->total_dof;
    const int n = b->n_inst;
    if (hipMalloc(&btil, sizeof(double) * tot) != hipSuccess || hipMalloc(&r, sizeof(double) * tot) != hipSuccess ||
        hipMalloc(&z, sizeof(double) * tot) != hipSuccess || hipMalloc(&norms, sizeof(double) * 2 * n) != hipSuccess ||
        hipMalloc(&part, sizeof(double) * (size_t)n * std::max(1, sp.max_chunks())) != hipSuccess ||
        hipMalloc(&act, sizeof(int32_t) * n) != hipSuccess)
      return RTE_ENOMEM;
    return RTE_OK;
  }
  void release() {
    sp.release();
    for (void* p : {(void*)btil, (void*)r, (void*)z, (void*)norms, (void*)part, (void*)act}) (void)hipFree(p);
    btil = r = z = norms = part = nullptr;
    act = nullptr;
  }
};

static std::vector<std::pair<rte_batch*, SiWork*>> g_si;

static SiWork* si_for(rte_batch* b) {
  for (auto& e : g_si)
    if (e.first == b) return e.second;
  auto* w = new SiWork();
  if (w->init(b) != RTE_OK) {
    w->release();
    delete w;
    return nullptr;
  }
  g_si.push_back({b, w});
  return w;
}

void si_forget(rte_batch* b) {
  for (size_t i = 0; i < g_si.size();) {
    if (g_si[i].first == b) {
      g_si[i].second->release();
      delete g_si[i].second;
      g_si.erase(g_si.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace rte

using namespace rte;

extern "C" int si_solve(const rte_batch* cb, const double* sigma_t, const double* sigma_s, const double* G,
                        const double* inflow, const rte_solve_opts* opts, const rte_rom* rom, double* phi,
                        rte_solve_stats* stats, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !sigma_t || !sigma_s || !G || !opts || !phi || !stats) return RTE_EINVAL;
  const rte_solve_opts& o = *opts;
  if (o.max_cycles < 1 || !(o.rtol > 0.0) || (o.sweep_dtype != RTE_F32 && o.sweep_dtype != RTE_F64) ||
      (o.precond != RTE_PC_NONE && o.precond != RTE_PC_DSA && o.precond != RTE_PC_ROMSAD) || o.window < 0 ||
      o.dsa_inner_max < 1 || o.dsa_restart < 0 || o.dsa_restart > 500 ||
      (o.dsa_variant != RTE_DSA_FC && o.dsa_variant != RTE_DSA_PC) ||
      (o.dsa_variant == RTE_DSA_PC && o.dsa_restart == 0))
    return RTE_EINVAL;
  if (o.precond == RTE_PC_ROMSAD && (!rom || !rom_matches(rom, b))) return RTE_EINVAL;
  if (b->n_fields > 0) return RTE_EINVAL;  // cross sections varying inside cells: FGMRES only
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RTE_TRY(validate_cross_sections(b, sigma_t, sigma_s, s));
  SiWork* w = si_for(b);
  if (!w) return RTE_ENOMEM;
  const int n = b->n_inst;
  const int prec = o.sweep_dtype == RTE_F32 ? 1 : 0;
  RTE_TRY(autotune_sweep(b, 0, sigma_t, s, sigma_s));
  if (prec == 1) RTE_TRY(autotune_sweep(b, 1, sigma_t, s, sigma_s));
  for (int q = 0; q < n; ++q) stats[q] = rte_solve_stats{};
  // b~ = T G~ (FP64) and its norm
  RTE_TRY(sweep_launch(b, 0, sigma_t, nullptr, nullptr, G, inflow, nullptr, s));
  RTE_TRY(reduce_partials(b, 0, 1.0, nullptr, 0.0, w->btil, s));
  RTE_TRY(knorm(w->sp, w->btil, w->part, w->norms, 1, nullptr, s));
  RTE_HIP(hipMemsetAsync(phi, 0, sizeof(double) * b->total_dof, s));
  std::vector<double> bn(n), rn(n);
  RTE_HIP(hipMemcpyAsync(bn.data(), w->norms, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  RTE_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> act(n);
  for (int q = 0; q < n; ++q) {
    stats[q].sweeps_f64 = 1;
    act[q] = bn[q] > 0.0 ? 1 : 0;
    stats[q].status = act[q] ? RTE_WNOTCONV : RTE_OK;
  }
  bool dsa_prepared = false;
  for (int l = 1; l <= o.max_cycles + 1; ++l) {
    RTE_HIP(hipMemcpyAsync(w->act, act.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    // r = b~ - A~ phi = T Sigma_s phi - phi + b~
    if (l == 1) {
      RTE_TRY(kcopy(w->sp, w->btil, w->r, w->act, s));
    } else {
      RTE_TRY(sweep_launch(b, prec, sigma_t, sigma_s, phi, nullptr, nullptr, nullptr, s, w->act,
                           batch_cell_ordinates(b, act.data())));
      RTE_TRY(reduce_partials(b, prec, 1.0, phi, -1.0, w->r, s, w->act, w->btil, 1.0));
      for (int q = 0; q < n; ++q)
        if (act[q]) (prec ? stats[q].sweeps_f32 : stats[q].sweeps_f64) += 1;
    }
    RTE_TRY(knorm(w->sp, w->r, w->part, w->norms + n, 1, w->act, s));
    RTE_HIP(hipMemcpyAsync(rn.data(), w->norms + n, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int q = 0; q < n; ++q) {
      if (!act[q]) continue;
      const double rel = rn[q] / bn[q];
      stats[q].true_relres = rel;
      stats[q].est_relres = rel;
      if (rel <= o.rtol) {
        act[q] = 0;
        stats[q].status = RTE_OK;
      }
      any = any || act[q];
    }
    if (!any || l > o.max_cycles) break;
    RTE_HIP(hipMemcpyAsync(w->act, act.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    // z = M_l^{-1} r
    int kind = o.precond;
    if (kind == RTE_PC_ROMSAD && l > o.window) kind = RTE_PC_DSA;
    if (kind == RTE_PC_NONE) {
      RTE_TRY(kcopy(w->sp, w->r, w->z, w->act, s));
    } else if (kind == RTE_PC_DSA) {
      RTE_TRY(dsa_apply(b, sigma_t, sigma_s, w->r, w->z, o.dsa_inner_tol, o.dsa_inner_max, o.dsa_restart, w->act,
                        nullptr, s, !dsa_prepared, o.dsa_variant));
      dsa_prepared = true;
    } else {
      const int st = romsad_apply_internal(rom, b, sigma_t, sigma_s, w->r, w->z, w->act, s);
      if (st != RTE_OK && st != RTE_ESINGULAR) return st;
    }
    RTE_TRY(kaxpby(w->sp, 1.0, w->z, 1.0, phi, w->act, s));
    for (int q = 0; q < n; ++q) {
      if (!act[q]) continue;
      stats[q].iterations += 1;
      stats[q].cycles = 1;
      if (kind == RTE_PC_DSA) stats[q].pc_dsa += 1;
      else if (kind == RTE_PC_ROMSAD) stats[q].pc_rom += 1;
    }
  }
  int ret = RTE_OK;
  for (int q = 0; q < n; ++q)
    if (stats[q].status != RTE_OK) ret = RTE_WNOTCONV;
  return ret;
}
