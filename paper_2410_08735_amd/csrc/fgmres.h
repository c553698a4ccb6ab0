// Batched flexible GMRES driver (Alg. 1).
#pragma once
#include "rom.h"

namespace rte {

struct SolveCtx {
  const rte_solve_opts* opts;
  const double *sigma_t, *sigma_s, *G, *inflow;
  const rte_rom* rom;
  const rte_mlp* mlp;
  const double* mu;
  int mu_dim;
  const int32_t* init_active;  // device mask of instances to solve (nullable = all)
  int keep;                    // record cycle 0's first `keep` Krylov vectors
};

// A captured operator application w = z - T Sigma_s z (sweep + reduction) for
// one Krylov index, replayed while its arguments and the sweep plan stay the same.
struct OpGraph {
  hipGraphExec_t exec = nullptr;
  const void* key[4] = {nullptr, nullptr, nullptr, nullptr};  // sigma_t, sigma_s, z, w
  int prec = -1, G = 0, threads = 0, variant = -1, opl = 0;
  bool reduce = true;  // the partial-flux reduction is part of the graph
  uint64_t gen = 0;  // the batch's plan / partial-buffer generation at capture
};

struct Fgmres {
  rte_batch* b = nullptr;
  std::vector<OpGraph> graphs;  // [prec * m + j]
  int m = 0;
  Krylov K;
  double *btil = nullptr, *r = nullptr, *bnorm = nullptr, *tolabs = nullptr, *rnorm = nullptr;
  int32_t *cyc = nullptr, *cyc_step = nullptr, *flags = nullptr;
  // instances whose reduced operator A_r(mu) is singular (DSA replaces the
  // ROM solve there), and the split of the activity mask by it
  int32_t *rsing = nullptr, *m_rom = nullptr, *m_dsa = nullptr;
  std::vector<int32_t> sing_h;
  bool any_sing = false;
  // pinned host copies of the activity mask after each Arnoldi step (two in
  // turn) and the events that mark them complete
  int32_t* mask_host = nullptr;
  hipEvent_t mask_ev[2] = {nullptr, nullptr};
  // pinned host staging of the per-solve and per-cycle reads and writes:
  // hd = [bnorm | rnorm | scal (8 per instance)], hi = [rsing | fail | the
  // mask after the cycle start | the cycle's mask | the cross-section check |
  // the learned correction's flags];
  // start_ev marks the cycle-start mask's copy complete
  double* hd = nullptr;
  int32_t* hi = nullptr;
  int32_t* xs_bad = nullptr;  // device: cross sections out of range somewhere
  hipEvent_t start_ev = nullptr;
  // the learned correction's fall-back flags of the last step, copied to
  // hi[4 n + 1 ..] behind it; flags_ev marks the copy complete
  hipEvent_t flags_ev = nullptr;
  bool flags_pending = false;
  int apply_flags(std::vector<int32_t>& which);
  // record of cycle 0 (xi recurrence): Z_0..Z_{w-1}, H block [(w+1) x w], beta
  double *recZ = nullptr, *recH = nullptr, *recBeta = nullptr, *recV = nullptr;
  int rec_w = 0;
  bool dsa_ready = false;
  std::vector<int32_t> rec_jdone;
  int init(rte_batch* b, int m);
  void release();
  void rec_release();
  int precondition(int jj, int cycle, const double* v, double* z, const SolveCtx& c, hipStream_t s,
                   std::vector<int32_t>& which);
  int solve(const SolveCtx& c, double* phi, rte_solve_stats* stats, hipStream_t s);
  int dsa_step(const double* v, double* z, const int32_t* mask, const SolveCtx& c, hipStream_t s);
  // reduce = false: the sweep only; the Arnoldi step then forms w from the
  // partial fluxes itself
  int apply_op(int j, int prec, const SolveCtx& c, bool use_graph, double units, hipStream_t s,
               bool reduce = true);
  void graphs_release();
};

Fgmres* fgmres_for(rte_batch* b, int m);
// Number of operator applications captured into HIP graphs so far (all batches).
int64_t graph_capture_count();
void fgmres_forget(rte_batch* b);

}  // namespace rte
