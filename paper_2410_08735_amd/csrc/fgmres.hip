// Flexible GMRES (Alg. 1) over a batch of instances, restarted from FP64 true
// residuals (the flexible outer iteration acts as refinement for FP32 sweeps).
#include <algorithm>
#include <cmath>

#include "fgmres.h"

namespace rte {

int Fgmres::init(rte_batch* batch, int m_) {
  b = batch;
  m = m_;
  std::vector<int64_t> lens(b->n_inst);
  for (int k = 0; k < b->n_inst; ++k) lens[k] = rte_batch_ndof(b, k);
  RTE_TRY(K.init(lens, m, true));
  const int64_t tot = b->total_dof;
  const int n = b->n_inst;
  if (hipMalloc(&btil, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&r, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&bnorm, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&tolabs, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&rnorm, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&cyc, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&cyc_step, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&flags, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&rsing, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&m_rom, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&m_dsa, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&xs_bad, sizeof(int32_t)) != hipSuccess ||
      hipHostMalloc(&mask_host, sizeof(int32_t) * 2 * n) != hipSuccess ||
      hipHostMalloc(&hd, sizeof(double) * 10 * n) != hipSuccess ||
      hipHostMalloc(&hi, sizeof(int32_t) * (5 * n + 1)) != hipSuccess)
    return RTE_ENOMEM;
  for (auto& e : mask_ev) RTE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  RTE_HIP(hipEventCreateWithFlags(&start_ev, hipEventDisableTiming));
  RTE_HIP(hipEventCreateWithFlags(&flags_ev, hipEventDisableTiming));
  return RTE_OK;
}

// The learned correction's fall-backs of the last preconditioning step,
// copied behind it: instances that fell back count as ROMSAD (DSA where their
// reduced operator is singular).
int Fgmres::apply_flags(std::vector<int32_t>& which) {
  if (!flags_pending) return RTE_OK;
  flags_pending = false;
  RTE_HIP(hipEventSynchronize(flags_ev));
  const int32_t* fb = hi + 4 * b->n_inst + 1;
  for (int q = 0; q < b->n_inst; ++q)
    if (fb[q]) which[q] = (any_sing && sing_h[q]) ? RTE_PC_DSA : -RTE_PC_ROMSAD;
  return RTE_OK;
}

void Fgmres::release() {
  graphs_release();
  K.release();
  for (void* p : {(void*)btil, (void*)r, (void*)bnorm, (void*)tolabs, (void*)rnorm, (void*)cyc,
                  (void*)cyc_step, (void*)flags, (void*)rsing, (void*)m_rom, (void*)m_dsa, (void*)xs_bad})
    (void)hipFree(p);
  btil = r = bnorm = tolabs = rnorm = nullptr;
  cyc = cyc_step = flags = rsing = m_rom = m_dsa = xs_bad = nullptr;
  for (void* p : {(void*)mask_host, (void*)hd, (void*)hi})
    if (p) (void)hipHostFree(p);
  mask_host = nullptr;
  hd = nullptr;
  hi = nullptr;
  for (auto& e : mask_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  for (hipEvent_t* e : {&start_ev, &flags_ev}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  rec_release();
}

void Fgmres::graphs_release() {
  for (auto& g : graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

// w = z_j - T Sigma_s z_j into v_{j+1}: one batched sweep and the deterministic
// partial-flux reduction, which also leaves the chunk partials of <w, v_0> in
// K.partA for the first MGS projection (without reduce only the sweep: the
// register-resident Arnoldi step forms w from the sweep's partial fluxes).
// With use_graph the pair is captured once per
// (precision, j) into a HIP graph and replayed; a new capture is made when the
// cross-section arrays, the plan or the buffers change (the batch's generation
// counts every reallocation of the plan tables and the partial buffer, whose
// addresses the graph embeds).  The kernels read the activity mask from
// device memory, so a replay follows the current mask.
static int64_t g_graph_captures = 0;
int64_t graph_capture_count() { return g_graph_captures; }

int Fgmres::apply_op(int j, int prec, const SolveCtx& c, bool use_graph, double units, hipStream_t s,
                     bool reduce) {
  if (!use_graph) {
    RTE_TRY(sweep_launch(b, prec, c.sigma_t, c.sigma_s, K.z(j), nullptr, nullptr, nullptr, s, K.active, units));
    if (!reduce) return RTE_OK;
    return reduce_partials_dot(b, prec, -1.0, K.z(j), 1.0, K.v(j + 1), K.v(0), K.partA, K.sp.max_chunks(),
                               KCHUNK, s, K.active);
  }
  if ((int)graphs.size() < 2 * m) graphs.resize(2 * m);
  OpGraph& g = graphs[prec * m + j];
  const Plan& p = b->plan[prec];
  const void* key[4] = {c.sigma_t, c.sigma_s, K.z(j), K.v(j + 1)};
  const bool same = g.exec && g.prec == prec && g.G == p.G && g.threads == p.threads && g.variant == p.variant &&
                    g.opl == p.opl && g.reduce == reduce && g.gen == b->gen && std::equal(key, key + 4, g.key);
  if (!same) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    hipGraph_t graph = nullptr;
    RTE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    // no profiler events inside the capture; they are recorded around the launch
    int st = sweep_launch(b, prec, c.sigma_t, c.sigma_s, K.z(j), nullptr, nullptr, nullptr, s, K.active, -2.0);
    if (st == RTE_OK && reduce)
      st = reduce_partials_dot(b, prec, -1.0, K.z(j), 1.0, K.v(j + 1), K.v(0), K.partA, K.sp.max_chunks(),
                               KCHUNK, s, K.active);
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != RTE_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return st != RTE_OK ? st : RTE_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      return RTE_EHIP;
    }
    ++g_graph_captures;
    g.gen = b->gen;
    g.prec = prec;
    g.G = p.G;
    g.threads = p.threads;
    g.variant = p.variant;
    g.opl = p.opl;
    g.reduce = reduce;
    std::copy(key, key + 4, g.key);
  }
  const bool prof = prof_enabled();
  if (prof) prof_begin(prec == 0 ? PROF_SWEEP_F64 : PROF_SWEEP_F32, s);
  RTE_HIP(hipGraphLaunch(g.exec, s));
  if (prof) prof_end(prec == 0 ? PROF_SWEEP_F64 : PROF_SWEEP_F32, s, units);
  return RTE_OK;
}

void Fgmres::rec_release() {
  (void)hipFree(recZ);
  (void)hipFree(recH);
  (void)hipFree(recBeta);
  (void)hipFree(recV);
  recZ = recH = recBeta = recV = nullptr;
  rec_w = 0;
}

// q = G + Sigma_s phi on every DoF of the active instances (Sigma_s of the
// DoF's cell region): the source whose sweep gives T (G + Sigma_s phi), so that
// the true residual b~ - A~ phi = T (G + Sigma_s phi) - phi takes one sweep.
__global__ void k_source_plus(const InstDev* __restrict__ insts, const int32_t* __restrict__ region,
                              const double* __restrict__ sigma_s, int max_regions,
                              const double* __restrict__ G, const double* __restrict__ phi,
                              double* __restrict__ q, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const int ncell = I.nx * I.ny, nl = I.nloc;
  const double* __restrict__ ss = sigma_s + (int64_t)b * max_regions;
  const int32_t* __restrict__ reg = region + I.region_off;
  // a cell per thread: its region's sigma_s once, its DoFs as 16-byte pairs
  // where they are aligned
  const bool pairs = (nl & 1) == 0 && (I.dof_off & 1) == 0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
    const double sc = ss[reg[c]];
    const int64_t o = I.dof_off + (int64_t)c * nl;
    if (pairs) {
      for (int k = 0; k < nl; k += 2) {
        const double2 g = *reinterpret_cast<const double2*>(G + o + k);
        const double2 f = *reinterpret_cast<const double2*>(phi + o + k);
        *reinterpret_cast<double2*>(q + o + k) = make_double2(g.x + sc * f.x, g.y + sc * f.y);
      }
    } else {
      for (int k = 0; k < nl; ++k) q[o + k] = G[o + k] + sc * phi[o + k];
    }
  }
}

// bad = 1 if some instance has a sigma_t that is not finite and positive or a
// sigma_s that is not finite and non-negative in one of its regions.
__global__ void k_check_sigma(const InstDev* __restrict__ insts, int n, int max_regions,
                              const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                              int32_t* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * max_regions) return;
  const int k = (int)(e / max_regions), R = (int)(e % max_regions);
  if (R >= insts[k].n_regions) return;
  const double t = sigma_t[e], a = sigma_s[e];
  if (!(isfinite(t) && t > 0.0) || !(isfinite(a) && a >= 0.0)) atomicOr(bad, 1);
}

// cyc = active = the host's mask for this cycle (read from pinned host
// memory), and the learned-correction flags cleared.
__global__ void k_cycle_masks(int n, const int32_t* __restrict__ host_mask, int32_t* __restrict__ cyc,
                              int32_t* __restrict__ active, int32_t* __restrict__ flags) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t v = host_mask[q];
  cyc[q] = v;
  active[q] = v;
  flags[q] = 0;
}

__global__ void k_tolabs(int n, const double* __restrict__ bnorm, double rtol, double* __restrict__ tol) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) tol[b] = rtol * bnorm[b];
}

__global__ void k_copy_h(int n, const double* __restrict__ H, int m, double* __restrict__ out, int w,
                         const double* __restrict__ scal, double* __restrict__ beta) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  for (int i = 0; i <= w; ++i)
    for (int j = 0; j < w; ++j)
      out[((int64_t)b * (w + 1) + i) * w + j] = (j < m && i <= m) ? H[(int64_t)b * (m + 1) * m + (int64_t)i * m + j] : 0.0;
  beta[b] = scal[b * 8 + 0];
}

// The learned correction stalls when a step reduces the Givens estimate by
// less than half; that instance then uses ROMSAD for the rest of the window.
__global__ void k_stall_check(int n, const double* __restrict__ scal, const int32_t* __restrict__ was_active,
                              int32_t* __restrict__ off) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || !was_active[b] || off[b]) return;
  const double prev = scal[b * 8 + 5], est = scal[b * 8 + 2];
  if (prev > 0.0 && est > 0.5 * prev) off[b] = 1;
}

// Instances with a singular reduced operator take DSA where the ROM solve
// would run: m_dsa = active & sing & off (off = 1 when not given), m_rom =
// active & !m_dsa.
__global__ void k_split_singular(int n, const int32_t* __restrict__ active, const int32_t* __restrict__ sing,
                                 const int32_t* __restrict__ off, int32_t* __restrict__ m_rom,
                                 int32_t* __restrict__ m_dsa) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const int a = active[b];
  const int d = a && sing[b] && (!off || off[b]);
  m_dsa[b] = d;
  m_rom[b] = a && !d;
}

int Fgmres::precondition(int jj, int cycle, const double* v, double* z, const SolveCtx& c, hipStream_t s,
                         std::vector<int32_t>& which) {
  const rte_solve_opts& o = *c.opts;
  int kind = o.precond;
  const bool in_window = jj <= o.window && (o.window_cycles <= 0 || cycle < o.window_cycles);
  if ((kind == RTE_PC_ROMSAD || kind == RTE_PC_MLP) && (!in_window || !c.rom)) kind = RTE_PC_DSA;
  if (kind == RTE_PC_MLP && !c.mlp) kind = RTE_PC_ROMSAD;
  which.assign(b->n_inst, kind);
  switch (kind) {
    case RTE_PC_NONE:
      return kcopy(K.sp, v, z, K.active, s);
    case RTE_PC_DSA:
      return dsa_step(v, z, K.active, c, s);
    case RTE_PC_ROMSAD: {
      const int32_t* mr = K.active;
      if (any_sing) {
        hipLaunchKernelGGL(k_split_singular, dim3((b->n_inst + 63) / 64), dim3(64), 0, s, b->n_inst, K.active,
                           rsing, nullptr, m_rom, m_dsa);
        RTE_HIP(hipGetLastError());
        mr = m_rom;
      }
      // A_r(mu) was factorised by the singularity check at the start of this solve
      const int st = romsad_apply_internal(c.rom, b, c.sigma_t, c.sigma_s, v, z, mr, s, nullptr, nullptr, nullptr,
                                           true);
      if (st < 0 && st != RTE_ESINGULAR) return st;
      if (any_sing) {
        RTE_TRY(dsa_step(v, z, m_dsa, c, s));
        for (int q = 0; q < b->n_inst; ++q)
          if (sing_h[q]) which[q] = RTE_PC_DSA;
      }
      return RTE_OK;
    }
    case RTE_PC_MLP: {
      RTE_TRY(mlp_precond(c.mlp, c.rom, b, c.sigma_t, c.sigma_s, c.mu, c.mu_dim, v, z, K.active, s,
                          flags));
      if (any_sing) {  // a stalled instance whose ROM solve is singular takes DSA
        hipLaunchKernelGGL(k_split_singular, dim3((b->n_inst + 63) / 64), dim3(64), 0, s, b->n_inst, K.active,
                           rsing, flags, m_rom, m_dsa);
        RTE_HIP(hipGetLastError());
        RTE_TRY(dsa_step(v, z, m_dsa, c, s));
      }
      // who fell back, for the statistics: read when the step's mask is
      // (apply_flags), so the GPU does not wait for the host here
      RTE_HIP(hipMemcpyAsync(hi + 4 * b->n_inst + 1, flags, sizeof(int32_t) * b->n_inst, hipMemcpyDeviceToHost,
                             s));
      RTE_HIP(hipEventRecord(flags_ev, s));
      flags_pending = true;
      return RTE_OK;
    }
  }
  return RTE_EINVAL;
}

// z = M_DSA^{-1} v on the masked instances; the first application of a solve
// rebuilds the cross-section-dependent multigrid data for every instance.
int Fgmres::dsa_step(const double* v, double* z, const int32_t* mask, const SolveCtx& c, hipStream_t s) {
  const rte_solve_opts& o = *c.opts;
  const bool prep = !dsa_ready;
  dsa_ready = true;
  return dsa_apply(b, c.sigma_t, c.sigma_s, v, z, o.dsa_inner_tol, o.dsa_inner_max, o.dsa_restart, mask,
                   nullptr, s, prep, o.dsa_variant);
}

int Fgmres::solve(const SolveCtx& c, double* phi, rte_solve_stats* stats, hipStream_t s) {
  const rte_solve_opts& o = *c.opts;
  const int n = b->n_inst;
  const int pin = o.sweep_dtype == RTE_F32 ? 1 : 0;
  // The cross sections are checked on the host before a solve that tunes the
  // sweep plans (the autotuner sweeps with them); otherwise on the device,
  // the result read together with ||b~|| (one host synchronisation fewer).
  const bool tune = !b->plan[0].tuned || (pin == 1 && !b->plan[1].tuned);
  if (tune) {
    RTE_TRY(validate_cross_sections(b, c.sigma_t, c.sigma_s, s));
    RTE_TRY(autotune_sweep(b, 0, c.sigma_t, s, c.sigma_s));
    if (pin == 1) RTE_TRY(autotune_sweep(b, 1, c.sigma_t, s, c.sigma_s));
  } else {
    RTE_TRY(fill_i32(xs_bad, 1, 0, s));
    const int64_t ne = (int64_t)n * b->max_regions;
    hipLaunchKernelGGL(k_check_sigma, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, b->d_inst, n,
                       b->max_regions, c.sigma_t, c.sigma_s, xs_bad);
    RTE_HIP(hipGetLastError());
  }
  for (int q = 0; q < n; ++q) stats[q] = rte_solve_stats{};
  dsa_ready = false;  // the DSA hierarchy is rebuilt for this call's cross sections
  K.bt = o.breakdown_tol > 0.0 ? o.breakdown_tol : 1e-14;
  RTE_TRY(fill_i32(K.fail, n, 0, s));
  if (o.precond == RTE_PC_MLP) RTE_TRY(mlp_rom_diff_reset(b, s));
  // A_r(mu) depends on mu only: its singularity is decided once per solve
  any_sing = false;
  sing_h.assign(n, 0);
  const bool with_rom = (o.precond == RTE_PC_ROMSAD || o.precond == RTE_PC_MLP) && c.rom;
  if (with_rom) RTE_TRY(rom_singular_check(c.rom, b, c.sigma_t, c.sigma_s, rsing, s));  // read with ||b~||
  std::vector<int32_t> live(n, 1);
  if (c.init_active) {
    RTE_HIP(hipMemcpyAsync(live.data(), c.init_active, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
  }
  int32_t* h_cm = hi + 3 * n;  // the host's mask of a cycle, in pinned memory
  std::copy(live.begin(), live.end(), h_cm);
  RTE_HIP(hipMemcpyAsync(cyc, h_cm, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  // b~ = T G~ and ||b~||.  With FP32 sweeps b~ only starts the first cycle and
  // scales the stopping test, so an FP32 sweep suffices: every true residual
  // is formed in FP64 from its definition, T (G~ + Sigma_s phi) - phi, and the
  // restarts refine away b~'s rounding.  With FP64 sweeps b~ is FP64 and the
  // residual b~ - (phi - T Sigma_s phi).
  const bool f32_btil = o.sweep_dtype == RTE_F32;
  const int btil_prec = f32_btil ? 1 : 0;
  RTE_TRY(sweep_launch(b, btil_prec, c.sigma_t, nullptr, nullptr, c.G, c.inflow, nullptr, s, cyc,
                       f32_btil ? -2.0 : batch_cell_ordinates(b, live.data())));
  // b~ and the chunk partials of ||b~||^2 in one pass
  RTE_TRY(reduce_partials_dot(b, btil_prec, 1.0, nullptr, 0.0, btil, nullptr, K.partA, K.sp.max_chunks(), KCHUNK,
                              s, cyc));
  for (int q = 0; q < n; ++q)
    if (live[q]) (f32_btil ? stats[q].sweeps_f32 : stats[q].sweeps_f64) += 1;
  RTE_TRY(knorm_finish(K.sp, K.partA, bnorm, 1, cyc, s));
  hipLaunchKernelGGL(k_tolabs, dim3((n + 63) / 64), dim3(64), 0, s, n, bnorm, o.rtol, tolabs);
  RTE_TRY(kcopy(K.sp, btil, r, cyc, s));
  double* h_rn = hd + n;
  double* h_sc = hd + 2 * n;
  int32_t* h_fail = hi + n;
  int32_t* h_start = hi + 2 * n;
  RTE_HIP(hipMemcpyAsync(hd, bnorm, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  if (with_rom) RTE_HIP(hipMemcpyAsync(hi, rsing, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  if (!tune) RTE_HIP(hipMemcpyAsync(hi + 4 * n, xs_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  RTE_HIP(hipStreamSynchronize(s));
  if (!tune && hi[4 * n]) return RTE_EINVAL;  // nothing of the caller's written yet
  if (with_rom)
    for (int q = 0; q < n; ++q) {
      sing_h[q] = hi[q];
      if (sing_h[q]) {
        any_sing = true;
        stats[q].rom_singular = 1;
      }
    }
  const std::vector<double> bn(hd, hd + n);
  RTE_HIP(hipMemsetAsync(phi, 0, sizeof(double) * b->total_dof, s));
  std::vector<int32_t> conv(n, 0), stop(n, 0);  // stop: status code of a stopped instance
  for (int q = 0; q < n; ++q) {
    if (!live[q] || bn[q] == 0.0) {
      conv[q] = 1;
      stats[q].true_relres = 0.0;
    } else if (!std::isfinite(bn[q])) {
      stop[q] = RTE_ENONFINITE;
      stats[q].true_relres = bn[q];
    }
  }
  std::vector<int32_t> act(n), which;
  bool recorded = false;
  for (int cycle = 0; cycle < o.max_cycles; ++cycle) {
    std::vector<int32_t> cm(n);
    int n_live = 0;
    for (int q = 0; q < n; ++q) {
      cm[q] = (conv[q] || stop[q]) ? 0 : 1;
      n_live += cm[q];
    }
    if (!n_live) break;
    // every earlier reader of the pinned mask finished before the last host
    // synchronisation, so it can be rewritten here
    std::copy(cm.begin(), cm.end(), h_cm);
    hipLaunchKernelGGL(k_cycle_masks, dim3((n + 63) / 64), dim3(64), 0, s, n, h_cm, cyc, K.active, flags);
    RTE_HIP(hipGetLastError());
    // With FP32 sweeps a cycle ends once the Givens estimate is 1e-4 of its
    // start (FP32 operators cannot take it much below ~1e-6, and measured on
    // the 96^2 checkerboard family an earlier restart from the FP64 true
    // residual also saves iterations: 9.4 at 1e-4 against 9.8 at 1e-6).
    RTE_TRY(kstart(K, r, tolabs, s, pin ? 1e-4 : 0.0));
    flags_pending = false;
    for (int q = 0; q < n; ++q) stats[q].cycles += cm[q];
    // The device activity mask decides who iterates in each step.  The host
    // enqueues step j before it reads the mask step j - 1 left (copied to
    // pinned memory behind that step), so the GPU never idles on the read; a
    // step enqueued after the last instance converged finds nobody active.
    // Step 0 runs with the mask the cycle start left, read the same way.
    RTE_HIP(hipMemcpyAsync(h_start, K.active, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipEventRecord(start_ev, s));
    act = cm;
    const bool any0 = n_live > 0;
    const bool stall = o.precond == RTE_PC_MLP;
    for (int j = 0; j < m && any0; ++j) {
      const bool stall_j = stall && j + 1 <= o.window && (o.window_cycles <= 0 || cycle < o.window_cycles);
      if (stall_j)  // who is active in this step, for the stall check after it
        RTE_HIP(hipMemcpyAsync(cyc_step, K.active, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
      RTE_TRY(precondition(j + 1, cycle, K.v(j), K.z(j), c, s, which));
      // w = A~ z_j = z_j - T Sigma_s z_j (work units of the previous step's mask, corrected below);
      // the register-resident Arnoldi step forms w from the sweep's partial fluxes itself
      const bool fold = arnoldi_in_registers(K);
      RTE_TRY(apply_op(j, pin, c, o.use_graph != 0 && s != nullptr, batch_cell_ordinates(b, act.data()), s,
                       !fold));
      const int pslot = pin ? PROF_SWEEP_F32 : PROF_SWEEP_F64;
      const int pidx = prof_enabled() ? prof_last(pslot) : -1;
      if (fold) {
        const PartialSrc src{b->plan[pin].d_parts, b->d_part, pin, K.z(j)};
        RTE_TRY(arnoldi_mgs(K, j, s, false, &src));
      } else {
        RTE_TRY(arnoldi_mgs(K, j, s, true));  // apply_op left <w, v_0> in partA
      }
      if (stall_j) {
        hipLaunchKernelGGL(k_stall_check, dim3((n + 63) / 64), dim3(64), 0, s, n, K.scal, cyc_step, flags);
        RTE_HIP(hipGetLastError());
      }
      int32_t* mh = mask_host + (j & 1) * n;
      RTE_HIP(hipMemcpyAsync(mh, K.active, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
      RTE_HIP(hipEventRecord(mask_ev[j & 1], s));
      {  // the mask step j ran with, left by the cycle start (j = 0) or step j - 1
        RTE_HIP(hipEventSynchronize(j > 0 ? mask_ev[(j - 1) & 1] : start_ev));
        const int32_t* prev = j > 0 ? mask_host + ((j - 1) & 1) * n : h_start;
        bool any = false;
        for (int q = 0; q < n; ++q) {
          act[q] = prev[q];
          any = any || act[q];
        }
        if (!any) {
          if (pidx >= 0) prof_set_units(pslot, pidx, -1.0);
          break;
        }
        if (pidx >= 0) prof_set_units(pslot, pidx, batch_cell_ordinates(b, act.data()));
      }
      RTE_TRY(apply_flags(which));
      for (int q = 0; q < n; ++q) {
        if (!act[q]) continue;
        stats[q].iterations += 1;
        if (pin) stats[q].sweeps_f32 += 1; else stats[q].sweeps_f64 += 1;
        const int k = which[q];
        if (k == RTE_PC_DSA) stats[q].pc_dsa += 1;
        else if (k == RTE_PC_ROMSAD) stats[q].pc_rom += 1;
        else if (k == RTE_PC_MLP) stats[q].pc_mlp += 1;
        else if (k == -RTE_PC_ROMSAD) { stats[q].pc_rom += 1; stats[q].pc_fallback += 1; }
      }
    }
    if (c.keep && !recorded) {
      // keep cycle 0's preconditioned vectors and Hessenberg block for the xi recurrence
      rec_release();
      rec_w = std::min(c.keep, m);
      if (hipMalloc(&recZ, sizeof(double) * rec_w * b->total_dof) != hipSuccess ||
          hipMalloc(&recV, sizeof(double) * rec_w * b->total_dof) != hipSuccess ||
          hipMalloc(&recH, sizeof(double) * n * (rec_w + 1) * rec_w) != hipSuccess ||
          hipMalloc(&recBeta, sizeof(double) * n) != hipSuccess)
        return RTE_ENOMEM;
      RTE_HIP(hipMemcpyAsync(recZ, K.Z, sizeof(double) * rec_w * b->total_dof,
                             hipMemcpyDeviceToDevice, s));
      RTE_HIP(hipMemcpyAsync(recV, K.V, sizeof(double) * rec_w * b->total_dof,
                             hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_copy_h, dim3((n + 63) / 64), dim3(64), 0, s, n, K.H, m, recH, rec_w,
                         K.scal, recBeta);
      RTE_HIP(hipMemcpyAsync(rec_jdone.data(), K.jdone, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
      recorded = true;
    }
    // phi += Z y ; r = b~ - A~ phi in FP64
    RTE_TRY(kylov_solve_update(K, K.Z, phi, s));
    if (f32_btil) {
      if (b->n_fields > 0) {  // q = G + Sigma_s phi with the cells' full scattering blocks
        RTE_TRY(kcopy(K.sp, c.G, r, cyc, s));
        RTE_TRY(field_apply(b, c.sigma_s, phi, r, true, cyc, s));
      } else {
        int max_cells = 0;
        for (const auto& I : b->inst) max_cells = std::max(max_cells, I.nx * I.ny);
        hipLaunchKernelGGL(k_source_plus, dim3(std::min((max_cells + 255) / 256, 1024), n), dim3(256), 0, s,
                           b->d_inst, b->d_region, c.sigma_s, b->max_regions, c.G, phi, r, cyc);
        RTE_HIP(hipGetLastError());
      }
      RTE_TRY(sweep_launch(b, 0, c.sigma_t, nullptr, nullptr, r, c.inflow, nullptr, s, cyc,
                           batch_cell_ordinates(b, cm.data())));
      // r and the chunk partials of ||r||^2 in one pass
      RTE_TRY(reduce_partials_dot(b, 0, 1.0, phi, -1.0, r, nullptr, K.partA, K.sp.max_chunks(), KCHUNK, s, cyc));
      RTE_TRY(knorm_finish(K.sp, K.partA, rnorm, 1, cyc, s));
    } else {
      RTE_TRY(sweep_launch(b, 0, c.sigma_t, c.sigma_s, phi, nullptr, nullptr, nullptr, s, cyc,
                           batch_cell_ordinates(b, cm.data())));
      RTE_TRY(reduce_partials(b, 0, 1.0, btil, 1.0, r, s, cyc, phi, -1.0));
      RTE_TRY(knorm(K.sp, r, K.partA, rnorm, 1, cyc, s));
    }
    RTE_HIP(hipMemcpyAsync(h_rn, rnorm, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipMemcpyAsync(h_sc, K.scal, sizeof(double) * 8 * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipMemcpyAsync(h_fail, K.fail, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    const double* rn = h_rn;
    const double* sc = h_sc;
    const int32_t* fl = h_fail;
    bool all = true;
    for (int q = 0; q < n; ++q) {
      if (cm[q]) {
        stats[q].sweeps_f64 += 1;
        stats[q].true_relres = rn[q] / bn[q];
        stats[q].est_relres = sc[8 * q + 2] / bn[q];
        if (!std::isfinite(rn[q]) || fl[q] == KFAIL_NONFINITE) stop[q] = RTE_ENONFINITE;
        else if (stats[q].true_relres <= o.rtol) conv[q] = 1;
        else if (fl[q] == KFAIL_BREAKDOWN) stop[q] = RTE_EBREAKDOWN;
      }
      all = all && (conv[q] || stop[q]);
    }
    if (all) break;
  }
  int ret = RTE_OK;
  for (int q = 0; q < n; ++q) {
    stats[q].status = conv[q] ? RTE_OK : (stop[q] ? stop[q] : RTE_WNOTCONV);
    if (!conv[q]) ret = RTE_WNOTCONV;
  }
  if (o.precond == RTE_PC_MLP) {
    std::vector<double> jm;
    RTE_TRY(mlp_rom_diff_read(b, jm, s));
    for (int q = 0; q < n; ++q) stats[q].mlp_rom_diff = jm[q];
  }
  return ret;
}

struct FgCache {
  rte_batch* b;
  int m;
  Fgmres* f;
};
static std::vector<FgCache> g_fg;

Fgmres* fgmres_for(rte_batch* b, int m) {
  for (auto& c : g_fg)
    if (c.b == b && c.m == m) return c.f;
  auto* f = new Fgmres();
  f->rec_jdone.assign(b->n_inst, 0);
  if (f->init(b, m) != RTE_OK) {
    f->release();
    delete f;
    return nullptr;
  }
  g_fg.push_back({b, m, f});
  return f;
}

void fgmres_forget(rte_batch* b) {
  for (size_t i = 0; i < g_fg.size();) {
    if (g_fg[i].b == b) {
      g_fg[i].f->release();
      delete g_fg[i].f;
      g_fg.erase(g_fg.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace rte

extern "C" int fgmres_solve(const rte_batch* cb, const double* sigma_t, const double* sigma_s,
                            const double* G, const double* inflow, const rte_solve_opts* opts,
                            const rte_rom* rom, const rte_mlp* mlp, const double* mu, int mu_dim,
                            double* phi, rte_solve_stats* stats, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !sigma_t || !sigma_s || !G || !opts || !phi || !stats) return RTE_EINVAL;
  const rte_solve_opts& o = *opts;
  if (o.m < 1 || o.m > 500 || o.max_cycles < 1 || !(o.rtol > 0.0) ||
      (o.sweep_dtype != RTE_F32 && o.sweep_dtype != RTE_F64) || o.precond < RTE_PC_NONE ||
      o.precond > RTE_PC_MLP || o.window < 0 || o.dsa_inner_max < 1 || o.dsa_restart < 0 ||
      o.dsa_restart > 500 || (o.dsa_variant != RTE_DSA_FC && o.dsa_variant != RTE_DSA_PC) ||
      (o.dsa_variant == RTE_DSA_PC && o.dsa_restart == 0))
    return RTE_EINVAL;
  if ((o.precond == RTE_PC_ROMSAD || o.precond == RTE_PC_MLP) && !rom) return RTE_EINVAL;
  if (rom && !rte::rom_matches(rom, b)) return RTE_EINVAL;
  if (o.precond == RTE_PC_MLP && rom && rom->is_set()) return RTE_EINVAL;  // one network per ROM basis
  if (o.precond == RTE_PC_MLP && (!mlp || !mu || mu_dim < 1)) return RTE_EINVAL;
  // cross sections varying inside the cells: the DSA must be the exact solve
  // (its V-cycles use cell averages), and the learned correction is not offered
  if (b->n_fields > 0 && (o.precond == RTE_PC_MLP ||
                          ((o.precond == RTE_PC_DSA || o.precond == RTE_PC_ROMSAD) && o.dsa_restart < 1)))
    return RTE_EINVAL;
  if (!(o.breakdown_tol >= 0.0) || o.breakdown_tol >= 1e3) return RTE_EINVAL;
  rte::Fgmres* f = rte::fgmres_for(b, o.m);  // the solve checks the cross sections
  if (!f) return RTE_ENOMEM;
  rte::SolveCtx c{};
  c.opts = opts;
  c.sigma_t = sigma_t;
  c.sigma_s = sigma_s;
  c.G = G;
  c.inflow = inflow;
  c.rom = rom;
  c.mlp = mlp;
  c.mu = mu;
  c.mu_dim = mu_dim;
  return f->solve(c, phi, stats, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int64_t rte_graph_captures(void) { return rte::graph_capture_count(); }
